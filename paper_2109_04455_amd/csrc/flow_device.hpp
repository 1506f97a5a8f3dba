// Per-node device code of the D2Q9 flow step, shared by the single-lattice
// and the batched kernels.  Populations are stored as Real; the node update
// computes in Acc (FP64 by default, so FP32 storage rounds once per store).
#pragma once

#include "stencil.hpp"

namespace lbf {
namespace flow {

// D2Q9 velocities: rest, E, N, W, S, NE, NW, SW, SE
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

template <typename Real>
__device__ __forceinline__ Real wgt(int i)
{
    return i == 0 ? Real(4) / Real(9) : (i < 5 ? Real(1) / Real(9) : Real(1) / Real(36));
}

template <typename Real>
__device__ __forceinline__ Real inlet_u(int y, int ny, double u0)
{
    const double h = ny - 2.0;
    return Real(4.0 * u0 * (y - 0.5) * (ny - 1.5 - y) / (h * h));
}

// Collide the shifted populations h in place; returns (u, v) and writes them.
// f_eq - w = w (drho + rho X) with X = 3 cu + 4.5 cu^2 - 1.5 u.u.  Opposite
// directions share the even part of X and differ in the sign of 3 cu, so each
// pair costs one evaluation.  Every product with rho = 1 + drho is formed as
// X + drho X, and 1/rho as 1 + d with d = -drho/(1 + drho): in FP32 the
// rounding of 1 + drho itself is then never used.  (drho changes by less
// than an ulp of 1 between neighbouring nodes, so that rounding error is
// smooth in space and would bias the steady state.)
template <typename Real>
__device__ __forceinline__ void collide(Real (&h)[9], Real omega, Real &u, Real &v)
{
    const Real drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const Real jx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
    const Real jy = (h[2] - h[4]) + (h[5] - h[8]) + (h[6] - h[7]);
    const Real d = -drho / (Real(1) + drho);
    u = jx + jx * d;
    v = jy + jy * d;
    const Real uu = Real(1.5) * (u * u + v * v);
    Real eq[9];
    eq[0] = wgt<Real>(0) * (drho - (uu + drho * uu));
    // cu per pair (direction, opposite): (E, W) u; (N, S) v; (NE, SW) u + v; (NW, SE) v - u
    const Real cu[4] = {u, v, u + v, v - u};
    const int dir[4] = {1, 2, 5, 6}, opp[4] = {3, 4, 7, 8};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const Real w = wgt<Real>(dir[q]);
        const Real xe = Real(4.5) * cu[q] * cu[q] - uu;
        const Real xo = Real(3) * cu[q];
        const Real even = drho + (xe + drho * xe);
        const Real odd = xo + drho * xo;
        eq[dir[q]] = w * (even + odd);
        eq[opp[q]] = w * (even - odd);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] -= omega * (h[i] - eq[i]);
}

// Byte offset of the source of population i of fluid node (x, id) with mask
// m in the previous lattice: half-way bounce-back reads the node's own
// opposite population, else population i of node id - c_i.  Populations
// entering through the open columns (x - c_i outside the lattice) are filled
// by Zou-He; their offset is the node's own slot, and `open` says so.
template <typename Off>
__device__ __forceinline__ Off source_off(int i, int x, int nx, int nxp, unsigned m, Off o, Off PB,
                                          Off B, bool &open)
{
    const int sx = x - CX[i];
    open = sx < 0 || sx >= nx;
    const bool wall = i != 0 && ((m >> (OPP[i] - 1)) & 1u);
    const Off back = (Off)(ptrdiff_t)(CX[i] + CY[i] * nxp) * B;  // modular
    return open ? o + i * PB : (wall ? o + OPP[i] * PB : o + i * PB - back);
}

// Zou-He rules at the open columns: velocity inlet at x = 0, pressure outlet
// at x = nx - 1 (nx >= 8, so at most one applies; two separate tests keep the
// compiler from merging the two branches' stores into an indexed one, which
// it would place in scratch memory).
template <typename Real, typename Acc>
__device__ __forceinline__ void zou_he(const FlowArgs<Real> &a, int x, int y, Acc (&h)[9])
{
    if (x == 0) {
        // Zou-He velocity inlet, u = (u_in(y), 0): unknown E, NE, SE.
        // In shifted form the known sum f0+fN+fS+2(fW+fNW+fSW) is 1 + sum h.
        // rho - 1 = (S + ux)/(1 - ux) with S the known shifted sum, so that
        // rho ux = ux + (rho - 1) ux never rounds 1 + (rho - 1) on its own.
        const Acc ux = inlet_u<Acc>(y, a.ny, a.u0);
        const Acc S = h[0] + h[2] + h[4] + Acc(2) * (h[3] + h[6] + h[7]);
        const Acc drho = (S + ux) / (Acc(1) - ux);
        const Acc rux = ux + drho * ux;
        h[1] = h[3] + Acc(2) / Acc(3) * rux;
        h[5] = h[7] - Acc(0.5) * (h[2] - h[4]) + rux / Acc(6);
        h[8] = h[6] + Acc(0.5) * (h[2] - h[4]) + rux / Acc(6);
    }
    if (x == a.nx - 1) {
        // Zou-He pressure outlet, rho = 1, u_y = 0: unknown W, NW, SW
        const Acc ux = h[0] + h[2] + h[4] + Acc(2) * (h[1] + h[5] + h[8]);
        h[3] = h[1] - Acc(2) / Acc(3) * ux;
        h[6] = h[8] - Acc(0.5) * (h[2] - h[4]) - ux / Acc(6);
        h[7] = h[5] + Acc(0.5) * (h[2] - h[4]) - ux / Acc(6);
    }
}

// Boundary rules, collision and stores of fluid node (x, y) with gathered h.
template <typename Real, typename Acc, bool WRITE_U, bool NT, bool WIDE>
__device__ __forceinline__ void finish_node(const FlowArgs<Real> &a, int x, int y, size_t id,
                                            Acc (&h)[9])
{
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const size_t P = a.plane;
    const Off PB = (Off)P * B, o = (Off)id * B;
    zou_he(a, x, y, h);
    Acc u, v;
    collide(h, Acc(a.omega), u, v);
    if (WRITE_U) {
        a.u[id] = Real(u);
        a.u[P + id] = Real(v);
    }
    const PopBlock<Real, NT, WIDE> out(a.dst, 9 * PB);
#pragma unroll
    for (int i = 0; i < 9; ++i) out.store(o + i * PB, Real(h[i]));
}

// Gather of fluid node (x, id) with mask m from the lattice in HBM: the
// streamed populations (bounce-back at solid sources), 0 where a population
// enters through an open column (Zou-He fills it).  All nine loads are
// issued before any use (an open source reads the node's own slot): no wait
// per direction.
template <typename Real, typename Acc, bool NT, bool WIDE>
__device__ __forceinline__ void gather_node(const FlowArgs<Real> &a, int x, size_t id, unsigned m,
                                            Acc (&h)[9])
{
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const Off PB = (Off)a.plane * B, o = (Off)id * B;
    const PopBlock<Real, NT, WIDE> in(a.src, 9 * PB);
    Real r[9];
    bool open[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = in.load(source_off<Off>(i, x, a.nx, a.nxp, m, o, PB, B, open[i]));
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = open[i] ? Acc(0) : Acc(r[i]);
}

// Full update of node (x, y): gather (bounce-back, Zou-He), collide, store.
template <typename Real, typename Acc, bool WRITE_U, bool NT, bool WIDE>
__device__ __forceinline__ void node_update(const FlowArgs<Real> &a, int x, int y)
{
    const size_t id = (size_t)y * a.nxp + x;
    const unsigned m = a.mask9[id];
    if (m & MASK9_SOLID) return;
    Acc h[9];
    gather_node<Real, Acc, NT, WIDE>(a, x, id, m, h);
    finish_node<Real, Acc, WRITE_U, NT, WIDE>(a, x, y, id, h);
}

// Nodes (x, y) and (x, y + 1) in one thread: the loads of both are issued
// before either is collided, which hides the latency of the FP64 collision
// (two rows per thread: 73 -> 54 us per step on a 4096 x 1024 lattice; FP32
// arithmetic gains nothing).  The loads go out with the masks, not after
// them: every population is first read from its streaming source (the
// node's own slot where that source lies outside the lattice), and only
// nodes next to a wall read their bounce-back populations afterwards, so
// wavefronts away from walls wait for memory once.  A node that is solid or
// outside the lattice stores nothing.
template <typename Real, typename Acc, bool WRITE_U, bool NT, bool WIDE>
__device__ __forceinline__ void node_update2(const FlowArgs<Real> &a, int x, int y)
{
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const Off PB = (Off)a.plane * B;
    const PopBlock<Real, NT, WIDE> in(a.src, 9 * PB);
    bool valid[2];
    size_t ids[2];
    unsigned m[2];
    Real r[2][9];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int yk = y + k;
        valid[k] = yk < a.ny;
        ids[k] = (size_t)(valid[k] ? yk : y) * a.nxp + x;
        m[k] = a.mask9[ids[k]];
        const Off o = (Off)ids[k] * B;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int sx = x - CX[i], sy = yk - CY[i];
            const bool inside = valid[k] && sx >= 0 && sx < a.nx && sy >= 0 && sy < a.ny;
            const Off back = (Off)(ptrdiff_t)(CX[i] + CY[i] * a.nxp) * B;  // modular
            r[k][i] = in.load(inside ? o + i * PB - back : o + i * PB);
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (!valid[k] || (m[k] & MASK9_SOLID)) continue;
        const Off o = (Off)ids[k] * B;
        if (m[k] & 0xFFu) {
            // half-way bounce-back: population i from the node's own opposite
#pragma unroll
            for (int i = 1; i < 9; ++i)
                if ((m[k] >> (OPP[i] - 1)) & 1u) r[k][i] = in.load(o + OPP[i] * PB);
        }
        Acc h[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int sx = x - CX[i];
            h[i] = (sx < 0 || sx >= a.nx) ? Acc(0) : Acc(r[k][i]);
        }
        finish_node<Real, Acc, WRITE_U, NT, WIDE>(a, x, y + k, ids[k], h);
    }
}

// Extended tile of the two-step flow launch: the shape of the ADR two-step
// tile (64 x (EY - 2) output nodes, one block of 64 (EY + 1) threads), so
// both launches share a grid.  FP32: 9 planes of 66 x 15 nodes, 36 KB of
// LDS, two 16-wavefront blocks per CU at <= 64 VGPRs; FP64: EY = 10.
template <typename Real>
struct FlowPairTile {
    static constexpr int EY = sizeof(Real) == 4 ? 15 : 10;
    static constexpr int OCC = sizeof(Real) == 4 ? 8 : 6;
    static constexpr int EX = 66, EP = EX * EY, TX = 64, TY = EY - 2;
};

// Two flow steps per launch (temporal blocking).  Step 1 updates every node
// of the extended tile (the output nodes and a ring of one node, corners
// included, which the diagonal populations reach) from the lattice in HBM
// and keeps the result in LDS, rounded to Real as a store would round it;
// step 2 gathers the output nodes from LDS, applies the same boundary rules
// and collision, and stores them (and their velocity with WRITE_U).  Sources
// a step-2 gather can reach are all in the tile: x +- 1 and y +- 1 of an
// output node; sources outside the lattice are never read (open columns are
// filled by Zou-He, rows outside the channel are walls).  Wavefront w < EY
// takes the 64 core nodes of extended row w in step 1 and output row w in
// step 2 (w < EY - 2); wavefront EY the two ring columns.
template <typename Real, typename Acc, bool WRITE_U, bool NT, bool WIDE>
__device__ __forceinline__ void pair_update(const FlowArgs<Real> &a, int bx, int by)
{
    using T = FlowPairTile<Real>;
    constexpr int EY = T::EY, EX = T::EX, EP = T::EP, TY = T::TY;
    __shared__ Real lds[9 * EP];
    __shared__ uint16_t lmask[EP];
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    {
        const int ey = w < EY ? w : lane >> 1;
        const int ex = w < EY ? lane + 1 : ((lane & 1) ? EX - 1 : 0);
        const int x = bx * 64 - 1 + ex, y = by * TY - 1 + ey;
        if (ey < EY && x >= 0 && x < a.nx && y >= 0 && y < a.ny) {
            const int e = ey * EX + ex;
            const size_t id = (size_t)y * a.nxp + x;
            // the loads go out with the mask: every population from its
            // streaming source (the node's own slot where that lies outside
            // the lattice), bounce-back populations reloaded only next to a
            // wall
            using Off = off_t_<WIDE>;
            constexpr Off B = sizeof(Real);
            const Off PB = (Off)a.plane * B, o = (Off)id * B;
            const PopBlock<Real, false, WIDE> in(a.src, 9 * PB);
            const unsigned m = a.mask9[id];
            Real r[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int sx = x - CX[i], sy = y - CY[i];
                const bool inside = sx >= 0 && sx < a.nx && sy >= 0 && sy < a.ny;
                const Off back = (Off)(ptrdiff_t)(CX[i] + CY[i] * a.nxp) * B;  // modular
                r[i] = in.load(inside ? o + i * PB - back : o + i * PB);
            }
            lmask[e] = (uint16_t)m;
            if (!(m & MASK9_SOLID)) {
                if (m & 0xFFu) {
#pragma unroll
                    for (int i = 1; i < 9; ++i)
                        if ((m >> (OPP[i] - 1)) & 1u) r[i] = in.load(o + OPP[i] * PB);
                }
                Acc h[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int sx = x - CX[i];
                    h[i] = (sx < 0 || sx >= a.nx) ? Acc(0) : Acc(r[i]);
                }
                zou_he(a, x, y, h);
                Acc u, v;
                collide(h, Acc(a.omega), u, v);
#pragma unroll
                for (int i = 0; i < 9; ++i) lds[i * EP + e] = Real(h[i]);
            }
        }
    }
    __syncthreads();
    if (w >= TY) return;
    const int x = bx * 64 + lane, y = by * TY + w;
    if (x >= a.nx || y >= a.ny) return;
    const int e = (w + 1) * EX + lane + 1;
    const unsigned m = lmask[e];
    if (m & MASK9_SOLID) return;
    Real r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sx = x - CX[i];
        const bool open = sx < 0 || sx >= a.nx;
        const bool wall = i != 0 && ((m >> (OPP[i] - 1)) & 1u);
        const int src = open ? i * EP + e : (wall ? OPP[i] * EP + e : i * EP + e - (CX[i] + CY[i] * EX));
        r[i] = lds[src];
    }
    Acc h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sx = x - CX[i];
        h[i] = (sx < 0 || sx >= a.nx) ? Acc(0) : Acc(r[i]);
    }
    finish_node<Real, Acc, WRITE_U, NT, WIDE>(a, x, y, (size_t)y * a.nxp + x, h);
}

}  // namespace flow
}  // namespace lbf
