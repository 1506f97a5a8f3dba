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

// Full update of node (x, y): gather (bounce-back, Zou-He), collide, store.
template <typename Real, typename Acc, bool WRITE_U, bool NT, bool WIDE>
__device__ __forceinline__ void node_update(const FlowArgs<Real> &a, int x, int y)
{
    const size_t id = (size_t)y * a.nxp + x;
    const unsigned m = a.mask9[id];
    if (m & MASK9_SOLID) return;
    const size_t P = a.plane;
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const Off PB = (Off)P * B, o = (Off)id * B;
    const PopBlock<Real, NT, WIDE> in(a.src, 9 * PB);
    Acc h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sx = x - CX[i];
        if (sx < 0 || sx >= a.nx) {
            h[i] = 0;  // open boundary: filled by Zou-He below
        } else {
            // half-way bounce-back reads the node's own opposite population,
            // else the population i of node id - c_i
            const bool wall = i != 0 && ((m >> (OPP[i] - 1)) & 1u);
            const Off back = (Off)(ptrdiff_t)(CX[i] + CY[i] * a.nxp) * B;  // modular
            h[i] = Acc(in.load(wall ? o + OPP[i] * PB : o + i * PB - back));
        }
    }
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
    } else if (x == a.nx - 1) {
        // Zou-He pressure outlet, rho = 1, u_y = 0: unknown W, NW, SW
        const Acc ux = h[0] + h[2] + h[4] + Acc(2) * (h[1] + h[5] + h[8]);
        h[3] = h[1] - Acc(2) / Acc(3) * ux;
        h[6] = h[8] - Acc(0.5) * (h[2] - h[4]) - ux / Acc(6);
        h[7] = h[5] + Acc(0.5) * (h[2] - h[4]) - ux / Acc(6);
    }
    Acc u, v;
    collide(h, Acc(a.omega), u, v);
    if (WRITE_U) {
        a.u[id] = Real(u);
        a.u[P + id] = Real(v);
    }
    {
        const PopBlock<Real, NT, WIDE> out(a.dst, 9 * PB);
#pragma unroll
        for (int i = 0; i < 9; ++i) out.store(o + i * PB, Real(h[i]));
    }
}

}  // namespace flow
}  // namespace lbf
