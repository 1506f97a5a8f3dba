// Per-node device code of the D2Q5 ADR step, shared by the single-lattice
// kernels and the batched (many-instance) kernels.
#pragma once

#include "stencil.hpp"

namespace lbf {
namespace adr {

// D2Q5: rest, E, N, W, S; w0 = 1/3, w1..4 = 1/6.
enum { DE = 1, DN = 2, DW = 3, DS = 4 };
constexpr unsigned BIT_E = 1u, BIT_N = 2u, BIT_W = 4u, BIT_S = 8u;

template <typename Real>
__device__ __forceinline__ Real w5(int i)
{
    return i == 0 ? Real(1) / Real(3) : Real(1) / Real(6);
}

// Gather the pre-collision (shifted) populations of one species at node
// (x, y) from the post-collision lattice `src` (base of this species).
template <typename Real, bool NT = false>
__device__ __forceinline__ void pull5(const Real *__restrict__ src, size_t P, size_t id, int x,
                                      int nx, int nxp, unsigned m, bool species_a, Real inlet_e,
                                      Real (&h)[5])
{
    h[0] = ld<NT>(src + id);
    // E arrives from x - 1
    if (x == 0)
        h[DE] = species_a ? inlet_e - ld<NT>(src + DW * P + id) : ld<NT>(src + DW * P + id);
    else if (m & BIT_W)
        h[DE] = ld<NT>(src + DW * P + id);
    else
        h[DE] = ld<NT>(src + DE * P + id - 1);
    // N arrives from y - 1
    h[DN] = (m & BIT_S) ? ld<NT>(src + DS * P + id) : ld<NT>(src + DN * P + id - nxp);
    // W arrives from x + 1
    if (x == nx - 1) {
        const Real sum = ld<NT>(src + id) + ld<NT>(src + DE * P + id) + ld<NT>(src + DN * P + id) +
                         ld<NT>(src + DW * P + id) + ld<NT>(src + DS * P + id);
        h[DW] = Real(2) * w5<Real>(DW) * sum - ld<NT>(src + DE * P + id);
    } else if (m & BIT_E) {
        h[DW] = ld<NT>(src + DE * P + id);
    } else {
        h[DW] = ld<NT>(src + DW * P + id + 1);
    }
    // S arrives from y + 1
    h[DS] = (m & BIT_N) ? ld<NT>(src + DN * P + id) : ld<NT>(src + DS * P + id + nxp);
}

// BGK collision of one species in shifted form (cref = 0 for B and C).
template <typename Real>
__device__ __forceinline__ void collide5(Real (&h)[5], Real delta, Real cref, const Real (&p)[5],
                                         Real omega)
{
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const Real w = w5<Real>(i);
        const Real target = w * p[i] * cref + w * (Real(1) + p[i]) * delta;
        h[i] -= omega * (h[i] - target);
    }
}

template <typename Real>
__device__ __forceinline__ void eq_factors(Real u, Real v, Real (&p)[5])
{
    const Real uu = Real(1.5) * (u * u + v * v);
    p[0] = -uu;
    p[DE] = Real(3) * u + Real(4.5) * u * u - uu;
    p[DN] = Real(3) * v + Real(4.5) * v * v - uu;
    p[DW] = -Real(3) * u + Real(4.5) * u * u - uu;
    p[DS] = -Real(3) * v + Real(4.5) * v * v - uu;
}

// Collide + react one node given its gathered populations (in place);
// records (C_A, C_B) at trace nodes when TRACE.
template <typename Real, int S, bool TRACE>
__device__ __forceinline__ void collide_react(const AdrArgs<Real> &a, size_t id, unsigned m, Real u,
                                              Real v, Real (&h)[S][5])
{
    Real p[5];
    eq_factors(u, v, p);
    Real c[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const Real delta = h[s][0] + h[s][1] + h[s][2] + h[s][3] + h[s][4];
        const Real cref = s == 0 ? a.cref : Real(0);
        c[s] = cref + delta;
        collide5(h[s], delta, cref, p, a.omega);
    }
    if (m & 0xF0u) {
        // link reaction (Eq. source_lbm): the population heading into a
        // catalytic node loses k w_i C_src, the product gains it
        const int off[5] = {0, 1, a.nxp, -1, -a.nxp};
#pragma unroll
        for (int i = 1; i < 5; ++i) {
            if (!((m >> (3 + i)) & 1u)) continue;
            const size_t sid = id + off[i];
            const Real k = a.kr[sid];
            if (a.type[sid] == 2) {
                const Real r = k * w5<Real>(i) * c[0];
                h[0][i] -= r;
                h[1][i] += r;
            } else if (S == 3) {
                const Real r = k * w5<Real>(i) * c[1];
                h[1][i] -= r;
                h[S - 1][i] += r;
            }
        }
        if (TRACE) {
            const int t = a.trace_idx[id];
            a.trace[2 * t] = c[0];
            a.trace[2 * t + 1] = S == 3 ? c[1] : Real(0);
        }
    }
}

// Collide + react + store for one node given its gathered populations.
template <typename Real, int S, bool TRACE, bool NT = false>
__device__ __forceinline__ void collide_react_store(const AdrArgs<Real> &a, size_t id, unsigned m,
                                                    Real (&h)[S][5])
{
    const size_t P = a.plane;
    collide_react<Real, S, TRACE>(a, id, m, a.ua[id], a.ua[P + id], h);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 5; ++i) st<NT>(a.dst + (s * 5 + i) * P + id, h[s][i]);
}

// Full update of node (x, y): gather, collide, react, store.
template <typename Real, int S, bool TRACE, bool NT>
__device__ __forceinline__ void node_update(const AdrArgs<Real> &a, int x, int y)
{
    const size_t id = (size_t)y * a.nxp + x;
    const unsigned m = a.mask5[id];
    if (m == MASK5_SOLID) return;
    const size_t P = a.plane;
    const Real inlet_e = Real(2) * w5<Real>(DE) * (a.cin - a.cref);
    Real h[S][5];
#pragma unroll
    for (int s = 0; s < S; ++s)
        pull5<Real, NT>(a.src + (size_t)s * 5 * P, P, id, x, a.nx, a.nxp, m, s == 0, inlet_e, h[s]);
    collide_react_store<Real, S, TRACE, NT>(a, id, m, h);
}

}  // namespace adr
}  // namespace lbf
