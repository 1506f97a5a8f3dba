// Internal declarations of the lattice-Boltzmann library: context layout,
// kernel argument blocks and the host-side launchers implemented next to
// their kernels.  Not part of the public ABI (include/lbf.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <tuple>

#include "lbf.h"

namespace lbf {

// Node-mask encodings -------------------------------------------------------
// D2Q5 mask (uint8), one per node:
//   bit d-1 (d = 1..4 for E, N, W, S): the neighbour x + c_d is not fluid
//           (solid node or outside the channel in y);
//   bit d+3: the neighbour x + c_d is a reacting catalyst for this species
//           count (type 2, or type 3 with three species).
//   A solid node holds MASK5_SOLID (impossible for a fluid node, whose
//   catalytic bits are a subset of its solid bits).
constexpr uint8_t MASK5_SOLID = 0xF0;
// D2Q9 mask (uint16): bit d-1 (d = 1..8): neighbour x + c_d not fluid;
// MASK9_SOLID marks a solid node.
constexpr uint16_t MASK9_SOLID = 0x8000;

// Rows are padded to a multiple of this many elements so each row starts on
// a 256-byte boundary (FP32) and wavefront accesses stay aligned.
constexpr int ROW_ALIGN = 64;

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Storage shift of species A: FP32 populations of A are stored as
// g_i - w_i c_in unless flags bit 2 asks for the plain values.
inline double storage_shift(const lbf_params &p)
{
    return (p.real_bytes == 4 && !(p.flags & 4)) ? p.c_in : 0.0;
}

// Steady-state test of one convergence check of an ADR run: eps moved by at
// most tol of itself since the previous check, the outflux of the last
// species is positive, and the outlet fluxes balance the inflow of A within
// MASS_BALANCE_TOL of it.  A steady state has nothing accumulating, so the
// fluxes through every cross-section equal the inflow; the two extra
// conditions reject the quiet phase before a front reaches the flux plane,
// when eps is 0 (or unchanged) at consecutive checks.  N: the ns outlet
// fluxes, prev: eps at the previous check (NaN at the first).
constexpr double MASS_BALANCE_TOL = 1e-3;
inline bool steady_check(const double *N, int ns, double inflow, double eps, double prev,
                         double tol)
{
    if (!(tol > 0) || std::isnan(prev) || std::isnan(eps) || !(N[ns - 1] > 0)) return false;
    double tot = 0;
    for (int s = 0; s < ns; ++s) tot += N[s];
    if (!(std::fabs(tot - inflow) <= MASS_BALANCE_TOL * std::fabs(inflow))) return false;
    return std::fabs(eps - prev) <= tol * std::fabs(eps);
}

// Launch shape shared by the stencil kernels: tiles of tx * ty nodes, with an
// optional XCD-aware renumbering of blocks (consecutive tiles land on the
// same XCD so that halo cache lines are shared within one L2).
struct Launch {
    int tx = 64, ty = 4;
    int gx = 1, gy = 1;
    bool xcd_remap = true;
    bool vec = false;  // ADR step: V nodes per thread (tile covers tx*V nodes in x)
    bool nontemporal = false;  // streaming loads/stores for the populations
    bool fp32_math = false;    // FP32 storage: compute in FP32 instead of FP64
    int mode = 0;              // ADR reaction: 0 links, 1 all populations next to catalysts
    bool periodic = false;     // ADR lattice periodic in x and y (no inlet / outlet)
    bool wide = true;          // 64-bit population offsets (a 9-plane lattice >= 4 GiB)
    dim3 grid() const { return dim3(gx * gy, 1, 1); }
    dim3 block() const { return dim3(tx * ty, 1, 1); }
};

template <typename Real>
struct FlowArgs {
    const Real *src;
    Real *dst;
    const uint16_t *mask9;
    Real *u;            // [2][plane] velocity output (only when written)
    int nx, ny, nxp;
    size_t plane;
    double omega;       // 1 / tau_f
    double u0;
    Launch L;
};

template <typename Real>
struct AdrArgs {
    const Real *src;    // post-collision state of the previous step [S][5][plane]
    Real *dst;          // post-collision state of this step
    const Real *ua;     // [2][plane] ADR velocity (already scaled)
    const uint8_t *mask5;
    const uint8_t *type;
    const Real *kr;     // per-node rate (read at catalytic neighbours)
    const int32_t *trace_idx;  // per-node index into the trace list
    Real *trace;        // [ntrace][2] concentrations (C_A, C_B) of this step (or NULL)
    Real *trace2;       // two-step launches: the same for the second step (or NULL)
    int nx, ny, nxp;
    size_t plane;
    double omega;       // 1 / tau_g
    double cin;         // inlet concentration of A
    double cref;        // storage shift of species A (populations stored as g - w_i cref)
    Launch L;
};



// launchers (return hipError_t of the launch)
hipError_t launch_masks(const uint8_t *type_in, uint8_t *type_pad, uint8_t *mask5, uint16_t *mask9,
                        int nx, int ny, int nxp, int nspecies, bool periodic, hipStream_t s);
hipError_t launch_production(int real_bytes, int ns, const AdrArgs<float> &af,
                             const AdrArgs<double> &ad, double *partial, int nblocks, double *out,
                             hipStream_t s);
hipError_t launch_totals(int real_bytes, int ns, const AdrArgs<float> &af, const AdrArgs<double> &ad,
                         double *partial, int nblocks, double *out, hipStream_t s);
hipError_t launch_trace_list(const uint8_t *mask5, int32_t *trace_idx, int32_t *trace_nodes,
                             int *counter, int nx, int ny, int nxp, hipStream_t s);
hipError_t launch_copy_rates(const double *k_in, const uint8_t *type_pad, void *kr, int real_bytes,
                             int nx, int ny, int nxp, hipStream_t s);

hipError_t launch_flow_init(int real_bytes, const FlowArgs<float> &af, const FlowArgs<double> &ad,
                            hipStream_t s);
hipError_t launch_flow_step(int real_bytes, bool write_u, const FlowArgs<float> &af,
                            const FlowArgs<double> &ad, hipStream_t s);
hipError_t launch_du_max(int real_bytes, const void *u, void *uprev, const uint16_t *mask9,
                         size_t n2, double *partial, int nblocks, double *out, hipStream_t s);

hipError_t launch_du_max_partials(const double *partial, int n, double *out, hipStream_t s);
hipError_t launch_velocity_handoff(int real_bytes, const void *u, void *ua, const uint8_t *mask5,
                                   double vel_scale, size_t plane, hipStream_t s);
hipError_t launch_adr_init(int real_bytes, int ns, const AdrArgs<float> &af,
                           const AdrArgs<double> &ad, hipStream_t s);
// Two ADR steps in one launch (temporal blocking through LDS); the argument
// blocks carry the launch of pair_tile's tile shape and, optionally, the
// trace slots of the two steps (trace, trace2).
hipError_t launch_adr_pair(int real_bytes, int ns, const AdrArgs<float> &af,
                           const AdrArgs<double> &ad, hipStream_t s);
void pair_tile(int real_bytes, int &tx, int &ty);
// Two ADR steps per launch by wavefronts marching along y (FP32 storage,
// FP64 arithmetic, link reactions in a channel, 32-bit offsets, no trace).
Launch march_launch(const Launch &base, int nx, int ny, int strip_rows);
hipError_t launch_adr_march(int ns, const AdrArgs<float> &a, hipStream_t s);
hipError_t launch_adr_step(int real_bytes, int ns, bool trace, const AdrArgs<float> &af,
                           const AdrArgs<double> &ad, hipStream_t s);
hipError_t launch_flux(int real_bytes, int ns, const void *src, const uint8_t *mask5, int nx, int ny,
                       int nxp, size_t plane, int xf, double cin, double cref, double *out,
                       hipStream_t s);
hipError_t launch_concentration(int real_bytes, int ns, int species, const AdrArgs<float> &af,
                                const AdrArgs<double> &ad, void *out, hipStream_t s);
hipError_t launch_trace_conc(int real_bytes, int ns, const AdrArgs<float> &af,
                             const AdrArgs<double> &ad, const int32_t *trace_nodes, int ntrace,
                             hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, size_t nbytes, hipStream_t s);
hipError_t launch_unpad(int real_bytes, const void *src, void *dst, int nx, int ny, int nxp,
                        hipStream_t s);
hipError_t launch_pad(int real_bytes, const void *src, void *dst, int nx, int ny, int nxp,
                      hipStream_t s);

}  // namespace lbf
