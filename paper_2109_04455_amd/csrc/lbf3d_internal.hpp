// Internal declarations and per-node device code of the 3D path: D3Q19 flow
// with a body force and D3Q7 ADR with link reactions.  Nodes are numbered row
// by row, a row being one (y, z) line of nxp >= nx nodes (x fastest), rows
// ordered row = z * ny + y; plane = nxp * ny * nz.  Node fields (masks,
// velocities) are plain [plane] arrays; populations use the segment layout
// of pidx below.
#pragma once

#include "lbf3d.h"
#include "stencil.hpp"

namespace lbf {
namespace d3 {

// D3Q19 in (+, -) pairs: rest; +-x, +-y, +-z; then the 12 edge directions.
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__host__ __device__ constexpr int opp19(int i) { return i == 0 ? 0 : (i & 1 ? i + 1 : i - 1); }

// D3Q19 mask (uint32): bit d-1 (d = 1..18): the neighbour x + c_d (periodic
// in x, y, z) is solid.  MASK19_SOLID marks a solid node.
constexpr uint32_t MASK19_SOLID = 1u << 31;
// D3Q7 mask (uint16): bit d-1 (d = 1..6 for +x, -x, +y, -y, +z, -z): the
// neighbour is solid (x outside [0, nx) is the open inlet/outlet, not
// solid); bit d+5: it is a reacting catalyst.  MASK7_SOLID marks a solid
// node (its bit 15 is never set for a fluid node).
constexpr uint16_t MASK7_SOLID = 0x8000;

struct Geo {
    int nx, ny, nz, nxp;
    size_t plane;
};

template <typename Real>
struct FlowArgs3 {
    const Real *src;
    Real *dst;
    const uint32_t *mask19;
    Real *u;            // [3][plane] velocity output (when written)
    Geo g;
    double omega;       // 1 / tau_f
    double fx;          // body force along x
    Launch L;
};

template <typename Real>
struct AdrArgs3 {
    const Real *src;    // post-collision state of the previous step (7 S populations)
    Real *dst;
    const Real *ua;     // [3][plane] ADR velocity
    const uint16_t *mask7;
    const uint8_t *type;
    const Real *kr;
    Geo g;
    double omega;
    double cin;
    double cref;        // storage shift of species A (g - w_i cref)
    Launch L;
};

// Population layout: the NQ populations of 64 consecutive nodes of a row are
// stored together (rows are padded to a multiple of 64 nodes, so a segment
// never straddles two rows).  A wavefront then finds all the populations of
// its 64 nodes in one block of NQ * 64 elements instead of in NQ planes far
// apart, which keeps the many row streams of a 3D stencil on few HBM pages.
constexpr int SEG = 64;
static_assert(ROW_ALIGN % SEG == 0, "segments must not straddle rows");

template <int NQ>
__device__ __forceinline__ size_t pidx(size_t node, int q)
{
    return ((node / SEG) * NQ + (size_t)q) * SEG + node % SEG;
}

// Byte offset of population 0 of `node` in a lattice of NQ populations of
// type Real (the layout of pidx); population q lies q * SEG * sizeof(Real)
// bytes further.
template <int NQ, typename Real, typename Off>
__device__ __forceinline__ Off seg_off(Off node)
{
    return ((node / SEG) * (Off)(NQ * SEG) + node % SEG) * (Off)sizeof(Real);
}

// Row index of (y + dy, z + dz), periodic in y and z (|dy|, |dz| <= 1).
__device__ __forceinline__ int row_of(const Geo &g, int y, int z, int dy, int dz)
{
    int yy = y + dy, zz = z + dz;
    yy = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
    zz = zz < 0 ? zz + g.nz : (zz >= g.nz ? zz - g.nz : zz);
    return zz * g.ny + yy;
}

hipError_t launch_masks3(const uint8_t *type_in, uint8_t *type_pad, uint16_t *mask7,
                         uint32_t *mask19, const Geo &g, int nspecies, hipStream_t s);
hipError_t launch_copy_rates3(const double *k_in, const uint8_t *type_pad, void *kr,
                              int real_bytes, const Geo &g, hipStream_t s);
hipError_t launch_flow_init3(int real_bytes, const FlowArgs3<float> &af,
                             const FlowArgs3<double> &ad, hipStream_t s);
hipError_t launch_flow_step3(int real_bytes, bool write_u, const FlowArgs3<float> &af,
                             const FlowArgs3<double> &ad, hipStream_t s);
hipError_t launch_du_max3(int real_bytes, const void *u, void *uprev, const uint32_t *mask19,
                          size_t plane, double *partial, int nblocks, double *out2,
                          hipStream_t s);
hipError_t launch_velocity_handoff3(int real_bytes, const void *u, void *ua,
                                    const uint16_t *mask7, size_t plane, double scale,
                                    hipStream_t s);
hipError_t launch_unpad3(int real_bytes, const void *src, void *dst, const Geo &g, hipStream_t s);
hipError_t launch_pad3(int real_bytes, const void *src, void *dst, const uint8_t *type_pad,
                       const Geo &g, hipStream_t s);
hipError_t launch_adr_init3(int real_bytes, int ns, const AdrArgs3<float> &af,
                            const AdrArgs3<double> &ad, hipStream_t s);
hipError_t launch_adr_step3(int real_bytes, int ns, const AdrArgs3<float> &af,
                            const AdrArgs3<double> &ad, hipStream_t s);
hipError_t launch_flux3(int real_bytes, int ns, const AdrArgs3<float> &af,
                        const AdrArgs3<double> &ad, int xf, double *out4, hipStream_t s);
hipError_t launch_concentration3(int real_bytes, int ns, int species, const AdrArgs3<float> &af,
                                 const AdrArgs3<double> &ad, void *out, hipStream_t s);
hipError_t launch_totals3(int real_bytes, int ns, const AdrArgs3<float> &af,
                          const AdrArgs3<double> &ad, double *partial, int nblocks, double *out,
                          hipStream_t s);

}  // namespace d3
}  // namespace lbf
