// Per-node device code of the D2Q5 ADR step, shared by the single-lattice
// kernels and the batched (many-instance) kernels.
//
// Populations are stored as Real (FP32 or FP64) and the arithmetic of a node
// update runs in Acc.  With FP32 storage the default Acc is FP64: each stored
// population is then rounded exactly once per step (at the store).  At a
// steady state the FP32 fixed point differs from the exact one by the
// per-step rounding residual times the residence time of the lattice, so
// fewer and unbiased roundings matter; the kernel is bandwidth-bound and the
// FP64 arithmetic costs no time.
#pragma once

#include "gather_src.hpp"
#include "stencil.hpp"

namespace lbf {
namespace adr {

// D2Q5: rest, E, N, W, S; w0 = 1/3, w1..4 = 1/6.
enum { DE = 1, DN = 2, DW = 3, DS = 4 };
constexpr unsigned BIT_E = 1u, BIT_N = 2u, BIT_W = 4u, BIT_S = 8u;

template <typename T>
__device__ __forceinline__ T w5(int i)
{
    return i == 0 ? T(1) / T(3) : T(1) / T(6);
}

// Gather the pre-collision (shifted) populations of one species at node
// (x, y) from a block of its 5 post-collision planes: plane d starts d PB
// bytes after the block base, rows are RB bytes apart and the node itself is
// at byte offset o.  A choice between two sources (bounce-back or
// neighbour) is a choice of offset.  Blk: PopBlock (lattice in HBM) or
// LdsBlock (a tile in LDS).  The five loads are issued together with
// offsets chosen by selects, and converted to Acc only after all of them:
// a branch per direction with the conversion inside would wait for each
// load in turn.  Inlet (x = 0): E comes from the node's own W (with the
// Dirichlet value for species A); outlet (x = nx - 1): W from the node's
// own populations (three more loads, outlet nodes only).
template <typename Acc, typename Blk, typename Off>
__device__ __forceinline__ void pull5_at(const Blk &blk, Off PB, Off RB, Off o, int x, int nx,
                                         unsigned m, bool species_a, Acc inlet_e, Acc (&h)[5])
{
    using R = typename Blk::real_type;
    constexpr Off B = sizeof(R);
    const Off oN = o + DN * PB, oW = o + DW * PB, oS = o + DS * PB;
    const bool in = x == 0, out = x == nx - 1;
    Off src[5];
    gather::adr_sources<Off>(B, PB, RB, o, x, nx, m, src);
    const R r0 = blk.load(src[0]), rE = blk.load(src[DE]), rN = blk.load(src[DN]),
            rW = blk.load(src[DW]), rS = blk.load(src[DS]);
    h[0] = Acc(r0);
    h[DE] = Acc(rE);
    h[DN] = Acc(rN);
    h[DW] = Acc(rW);
    h[DS] = Acc(rS);
    if (in && species_a) h[DE] = inlet_e - h[DE];
    if (out) {
        // rW is the node's own E here
        const Acc sum = h[0] + h[DW] + Acc(blk.load(oN)) + Acc(blk.load(oW)) + Acc(blk.load(oS));
        h[DW] = Acc(2) * w5<Acc>(DW) * sum - h[DW];
    }
}

// The same from the lattice in HBM: `src` is the base of this species, P the
// plane size in nodes, id the node index.
template <typename Real, typename Acc, bool NT, bool WIDE>
__device__ __forceinline__ void pull5(const Real *__restrict__ src, size_t P, size_t id, int x,
                                      int nx, int nxp, unsigned m, bool species_a, Acc inlet_e,
                                      Acc (&h)[5])
{
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const Off PB = (Off)P * B;
    const PopBlock<Real, NT, WIDE> blk(src, 5 * PB);
    pull5_at<Acc>(blk, PB, (Off)nxp * B, (Off)id * B, x, nx, m, species_a, inlet_e, h);
}

// Gather of all S species at one node: the source offsets are chosen once
// (they are the same for every species) and all 5 S loads are issued before
// any is converted to Acc, so a wavefront waits for memory once per gather.
// blk_of(s): the block of species s (PopBlock or LdsBlock).  Same results
// as pull5_at per species.
template <typename Acc, int S, typename BlkOf, typename Off>
__device__ __forceinline__ void pullS_at(const BlkOf &blk_of, Off PB, Off RB, Off o, int x,
                                         int nx, unsigned m, Acc inlet_e, Acc (&h)[S][5])
{
    using BlkT = decltype(blk_of(0));
    using R = typename BlkT::real_type;
    constexpr Off B = sizeof(R);
    const Off oN = o + DN * PB, oW = o + DW * PB, oS = o + DS * PB;
    const bool in = x == 0, out = x == nx - 1;
    Off src[5];
    gather::adr_sources<Off>(B, PB, RB, o, x, nx, m, src);
    R r[S][5];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const BlkT blk = blk_of(s);
#pragma unroll
        for (int i = 0; i < 5; ++i) r[s][i] = blk.load(src[i]);
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 5; ++i) h[s][i] = Acc(r[s][i]);
    if (in) h[0][DE] = inlet_e - h[0][DE];
    if (out) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            // h[s][DW] is the node's own E here
            const BlkT blk = blk_of(s);
            const Acc sum = h[s][0] + h[s][DW] + Acc(blk.load(oN)) + Acc(blk.load(oW)) +
                            Acc(blk.load(oS));
            h[s][DW] = Acc(2) * w5<Acc>(DW) * sum - h[s][DW];
        }
    }
}

// The same from the lattice in HBM: species s starts at src + s 5 P.
template <typename Real, typename Acc, int S, bool NT, bool WIDE>
__device__ __forceinline__ void pullS(const Real *__restrict__ src, size_t P, size_t id, int x,
                                      int nx, int nxp, unsigned m, Acc inlet_e, Acc (&h)[S][5])
{
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const Off PB = (Off)P * B;
    const auto blk_of = [&](int s) { return PopBlock<Real, NT, WIDE>(src + (size_t)s * 5 * P, 5 * PB); };
    pullS_at<Acc, S>(blk_of, PB, (Off)nxp * B, (Off)id * B, x, nx, m, inlet_e, h);
}

// Gather for a box periodic in x and y (no inlet or outlet); solid
// neighbours still bounce back.  nb[d] are the wrapped neighbour indices.
template <typename Real, typename Acc, bool NT>
__device__ __forceinline__ void pull5_periodic(const Real *__restrict__ src, size_t P, size_t id,
                                               const size_t (&nb)[5], unsigned m, Acc (&h)[5])
{
    // sources chosen by address, all five loads issued before any use
    const Real r0 = ld<NT>(src + id);
    const Real rE = ld<NT>((m & BIT_W) ? src + DW * P + id : src + DE * P + nb[DW]);
    const Real rN = ld<NT>((m & BIT_S) ? src + DS * P + id : src + DN * P + nb[DS]);
    const Real rW = ld<NT>((m & BIT_E) ? src + DE * P + id : src + DW * P + nb[DE]);
    const Real rS = ld<NT>((m & BIT_N) ? src + DN * P + id : src + DS * P + nb[DN]);
    h[0] = Acc(r0);
    h[DE] = Acc(rE);
    h[DN] = Acc(rN);
    h[DW] = Acc(rW);
    h[DS] = Acc(rS);
}

// Neighbour indices x + c_d of node (x, y), wrapped in x and y.
__device__ __forceinline__ void periodic_neighbours(int x, int y, int nx, int ny, int nxp,
                                                    size_t (&nb)[5])
{
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    nb[0] = (size_t)y * nxp + x;
    nb[DE] = (size_t)y * nxp + xp;
    nb[DN] = (size_t)yp * nxp + x;
    nb[DW] = (size_t)y * nxp + xm;
    nb[DS] = (size_t)ym * nxp + x;
}

// BGK collision of one species in shifted form: the equilibrium of
// population i is w_i p_i cref + w_i (1 + p_i) delta, written as
// off[i] + mul[i] delta with the per-node factors mul[i] = w_i (1 + p_i) and
// off[i] = w_i p_i cref computed once for all species (off = 0 for B and C,
// whose cref is 0).
template <typename Acc, bool OFF>
__device__ __forceinline__ void collide5(Acc (&h)[5], Acc delta, const Acc (&mul)[5],
                                         const Acc (&off)[5], Acc omega)
{
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const Acc target = OFF ? off[i] + mul[i] * delta : mul[i] * delta;
        h[i] -= omega * (h[i] - target);
    }
}

template <typename Acc>
__device__ __forceinline__ void eq_factors(Acc u, Acc v, Acc (&p)[5])
{
    const Acc uu = Acc(1.5) * (u * u + v * v);
    p[0] = -uu;
    p[DE] = Acc(3) * u + Acc(4.5) * u * u - uu;
    p[DN] = Acc(3) * v + Acc(4.5) * v * v - uu;
    p[DW] = -Acc(3) * u + Acc(4.5) * u * u - uu;
    p[DS] = -Acc(3) * v + Acc(4.5) * v * v - uu;
}

// Collide + react one node given its gathered populations (in place);
// records (C_A, C_B) at trace nodes when TRACE and a.trace is set.  MODE 0: link reaction, only
// the population heading into a catalytic node reacts (rate of that node);
// MODE 1: the paper's comparison variant, every population of a fluid node
// next to catalysts reacts, with the mean rate of its catalytic neighbours of
// each type.  nb: neighbour indices x + c_d (NULL: the unwrapped lattice).
template <typename Real, typename Acc, int S, bool TRACE, int MODE = 0>
__device__ __forceinline__ void collide_react(const AdrArgs<Real> &a, size_t id, unsigned m, Acc u,
                                              Acc v, Acc (&h)[S][5], const size_t *nb = nullptr)
{
    // FP64: h* = (1 - omega) h + omega feq with the per-node factors
    // mul = omega w (1 + p), off = omega w p cref (two operations per
    // population).  FP32 arithmetic keeps h - omega (h - feq) with
    // mul = w (1 + p): 1 + p_i together loses less of the small p_i.
    constexpr bool F64 = sizeof(Acc) == 8;
    const Acc om = Acc(a.omega);
    Acc mul[5], off[5];
    {
        Acc p[5];
        eq_factors(u, v, p);
        const Acc omc = om * Acc(a.cref);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const Acc w = w5<Acc>(i), wp = w * p[i];
            if constexpr (F64) {
                mul[i] = om * w + om * wp;
                off[i] = omc * wp;
            } else {
                mul[i] = w * (Acc(1) + p[i]);
                off[i] = wp * Acc(a.cref);
            }
        }
    }
    const Acc keep = Acc(1) - om;
    Acc c[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const Acc delta = h[s][0] + h[s][1] + h[s][2] + h[s][3] + h[s][4];
        c[s] = (s == 0 ? Acc(a.cref) : Acc(0)) + delta;
        if constexpr (F64) {
#pragma unroll
            for (int i = 0; i < 5; ++i)
                h[s][i] = keep * h[s][i] + (s == 0 ? mul[i] * delta + off[i] : mul[i] * delta);
        } else if (s == 0) {
            collide5<Acc, true>(h[s], delta, mul, off, om);
        } else {
            collide5<Acc, false>(h[s], delta, mul, off, om);
        }
    }
    if (m & 0xF0u) {
        const int off[5] = {0, 1, a.nxp, -1, -a.nxp};
        if (MODE == 0) {
            // Eq. source_lbm at the links: the population heading into a
            // catalytic node loses k w_i C_src, the product gains it.  The
            // rate and type of all four neighbours are loaded together (the
            // index clamped into the plane), then used where a link bit is set
            Real kv[5];
            uint8_t tv[5];
#pragma unroll
            for (int i = 1; i < 5; ++i) {
                const long j = (long)id + off[i];
                const size_t sid = nb ? nb[i] : (size_t)(j < 0 ? 0 : (j >= (long)a.plane ? (long)a.plane - 1 : j));
                kv[i] = a.kr[sid];
                tv[i] = a.type[sid];
            }
#pragma unroll
            for (int i = 1; i < 5; ++i) {
                if (!((m >> (3 + i)) & 1u)) continue;
                const Acc k = Acc(kv[i]);
                if (tv[i] == 2) {
                    const Acc r = k * w5<Acc>(i) * c[0];
                    h[0][i] -= r;
                    h[1][i] += r;
                } else if (S == 3) {
                    const Acc r = k * w5<Acc>(i) * c[1];
                    h[1][i] -= r;
                    h[S - 1][i] += r;
                }
            }
        } else {
            Acc ks[2] = {0, 0};
            int kc[2] = {0, 0};
#pragma unroll
            for (int i = 1; i < 5; ++i) {
                if (!((m >> (3 + i)) & 1u)) continue;
                const size_t sid = nb ? nb[i] : id + off[i];
                const int q = a.type[sid] == 2 ? 0 : 1;
                ks[q] += Acc(a.kr[sid]);
                kc[q] += 1;
            }
#pragma unroll
            for (int q = 0; q < 2 && q < S - 1; ++q) {
                if (kc[q] == 0) continue;
                const Acc kk = ks[q] / Acc(kc[q]);
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    const Acc r = kk * w5<Acc>(j) * c[q];
                    h[q][j] -= r;
                    h[q + 1][j] += r;
                }
            }
        }
        if (TRACE && a.trace) {
            const int t = a.trace_idx[id];
            a.trace[2 * t] = Real(c[0]);
            a.trace[2 * t + 1] = S == 3 ? Real(c[1]) : Real(0);
        }
    }
}

// Store the post-collision populations of node id.
template <typename Real, typename Acc, int S, bool NT, bool WIDE>
__device__ __forceinline__ void store_node(const AdrArgs<Real> &a, size_t id, const Acc (&h)[S][5])
{
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const Off PB = (Off)a.plane * B, o = (Off)id * B;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const PopBlock<Real, NT, WIDE> out(a.dst + (size_t)s * 5 * a.plane, 5 * PB);
#pragma unroll
        for (int i = 0; i < 5; ++i) out.store(o + i * PB, Real(h[s][i]));
    }
}

// Collide + react + store for one node given its gathered populations.
template <typename Real, typename Acc, int S, bool TRACE, bool NT, bool WIDE>
__device__ __forceinline__ void collide_react_store(const AdrArgs<Real> &a, size_t id, unsigned m,
                                                    Acc (&h)[S][5])
{
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const Off PB = (Off)a.plane * B, o = (Off)id * B;
    const PopBlock<Real, false, WIDE> vel(a.ua, 2 * PB);
    collide_react<Real, Acc, S, TRACE>(a, id, m, Acc(vel.load(o)), Acc(vel.load(o + PB)), h);
    store_node<Real, Acc, S, NT, WIDE>(a, id, h);
}

// Full update of node (x, y): gather, collide, react, store.
template <typename Real, typename Acc, int S, bool TRACE, bool NT, bool WIDE>
__device__ __forceinline__ void node_update(const AdrArgs<Real> &a, int x, int y)
{
    const size_t id = (size_t)y * a.nxp + x;
    const unsigned m = a.mask5[id];
    if (m == MASK5_SOLID) return;
    const size_t P = a.plane;
    const Acc inlet_e = Acc(2) * w5<Acc>(DE) * (Acc(a.cin) - Acc(a.cref));
    Acc h[S][5];
    pullS<Real, Acc, S, NT, WIDE>(a.src, P, id, x, a.nx, a.nxp, m, inlet_e, h);
    collide_react_store<Real, Acc, S, TRACE, NT, WIDE>(a, id, m, h);
}

// Node update for the reaction variant (MODE 1) and/or the periodic box,
// arithmetic in FP64.
template <typename Real, int S, bool NT, int MODE, bool PERIODIC>
__device__ __forceinline__ void node_update_ext(const AdrArgs<Real> &a, int x, int y)
{
    const size_t id = (size_t)y * a.nxp + x;
    const unsigned m = a.mask5[id];
    if (m == MASK5_SOLID) return;
    const size_t P = a.plane;
    double h[S][5];
    size_t nb[5];
    if (PERIODIC) {
        periodic_neighbours(x, y, a.nx, a.ny, a.nxp, nb);
#pragma unroll
        for (int s = 0; s < S; ++s)
            pull5_periodic<Real, double, NT>(a.src + (size_t)s * 5 * P, P, id, nb, m, h[s]);
    } else {
        const int off[5] = {0, 1, a.nxp, -1, -a.nxp};
#pragma unroll
        for (int d = 0; d < 5; ++d) nb[d] = id + off[d];
        const double inlet_e = 2.0 * w5<double>(DE) * (a.cin - a.cref);
        pullS<Real, double, S, NT, true>(a.src, P, id, x, a.nx, a.nxp, m, inlet_e, h);
    }
    collide_react<Real, double, S, false, MODE>(a, id, m, double(a.ua[id]), double(a.ua[P + id]),
                                                h, nb);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 5; ++i) st<NT>(a.dst + (s * 5 + i) * P + id, Real(h[s][i]));
}

// Extended tile of the two-step kernel: 66 x EY nodes around 64 x (EY - 2)
// output nodes.  EY = 15 for FP32 storage: 16 wavefronts and 58 KB of LDS per
// block, two blocks per CU when a wavefront holds at most 64 VGPRs (OCC = 8
// wavefronts per SIMD; one block per CU otherwise).  FP64: EY = 10, 11
// wavefronts and 77 KB, two blocks per CU (6 wavefronts per SIMD).  Measured
// on a 4096 x 1024 channel against EY = 6 .. 12 (FP32) and 4 .. 8 (FP64).
template <typename Real>
struct PairTile {
    static constexpr int EY = sizeof(Real) == 4 ? 15 : 10;
    static constexpr int OCC = sizeof(Real) == 4 ? 8 : 6;
    // masks and velocities of the tile in LDS too (FP32: 67 KB per block)
    static constexpr bool ULDS = sizeof(Real) == 4;
    // streaming hint on the step-1 loads
    static constexpr bool NTL = false;
    static constexpr int TX = 64, TY = EY - 2;  // output nodes per block
};

// LDS of one two-step tile: the step-1 populations of the extended tile and,
// with ULDS, its masks and velocities.
template <typename Real, int S>
struct PairLds {
    static constexpr int EY = PairTile<Real>::EY, EX = 66, EP = EX * EY;
    static constexpr bool ULDS = PairTile<Real>::ULDS;
    Real pop[5 * S * EP];
    Real vel[ULDS ? 2 * EP : 1];
    uint8_t mask[ULDS ? EP : 1];
};

// The extended-tile node a thread updates in step 1 of tile (bx, by):
// wavefront w < EY takes the 64 core nodes of extended row w, wavefront EY
// the two ring columns of every row.
struct PairNode {
    int ex, ey, x, y, e;
    bool inside;
    size_t id;
};

template <typename Real>
__device__ __forceinline__ PairNode pair_node(const AdrArgs<Real> &a, int bx, int by)
{
    constexpr int EY = PairTile<Real>::EY, EX = 66, TY = EY - 2;
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    PairNode n;
    if (w < EY) {
        n.ey = w;
        n.ex = lane + 1;
    } else {
        n.ey = lane >> 1;
        n.ex = (lane & 1) ? EX - 1 : 0;
    }
    n.x = bx * 64 - 1 + n.ex;
    n.y = by * TY - 1 + n.ey;
    n.inside = n.ey < EY && n.x >= 0 && n.x < a.nx && n.y >= 0 && n.y < a.ny;
    n.id = (size_t)(n.inside ? n.y : 0) * a.nxp + (n.inside ? n.x : 0);
    n.e = n.ey * EX + n.ex;
    return n;
}

// What step 1 of a node reads before its gather: mask and velocity.
template <typename Real>
struct PairPre {
    unsigned m;
    Real u, v;
};

template <typename Real, bool WIDE>
__device__ __forceinline__ PairPre<Real> pair_pre(const AdrArgs<Real> &a, const PairNode &n)
{
    PairPre<Real> q{MASK5_SOLID, Real(0), Real(0)};
    if (n.inside) {
        using Off = off_t_<WIDE>;
        constexpr Off B = sizeof(Real);
        const Off PB = (Off)a.plane * B, o = (Off)n.id * B;
        const PopBlock<Real, false, WIDE> vel(a.ua, 2 * PB);
        q.m = a.mask5[n.id];
        q.u = vel.load(o);
        q.v = vel.load(o + PB);
    }
    return q;
}

// Step 1 of a node into the LDS tile.
template <typename Real, typename Acc, int S, bool WIDE, bool TRACE>
__device__ __forceinline__ void pair_step1(PairLds<Real, S> &L, const AdrArgs<Real> &a,
                                           const PairNode &n, const PairPre<Real> &q)
{
    constexpr int EY = PairTile<Real>::EY, TY = EY - 2, EP = PairLds<Real, S>::EP;
    if (!n.inside) return;
    const size_t P = a.plane;
    if (PairLds<Real, S>::ULDS) L.mask[n.e] = (uint8_t)q.m;
    // solid nodes gather nothing: their mask has no bounce-back bits, so a
    // gather would read the neighbours' planes (past the last row of the
    // lattice for a node of the top wall row)
    if (q.m == MASK5_SOLID) {
        if (PairLds<Real, S>::ULDS) {
            L.vel[n.e] = q.u;
            L.vel[EP + n.e] = q.v;
        }
        return;
    }
    const Acc inlet_e = Acc(2) * w5<Acc>(DE) * (Acc(a.cin) - Acc(a.cref));
    Acc h[S][5];
    pullS<Real, Acc, S, PairTile<Real>::NTL, WIDE>(a.src, P, n.id, n.x, a.nx, a.nxp, q.m, inlet_e, h);
    if (PairLds<Real, S>::ULDS) {
        L.vel[n.e] = q.u;
        L.vel[EP + n.e] = q.v;
    }
    if constexpr (TRACE) {
        // step-1 concentrations are recorded by the block owning the node
        AdrArgs<Real> a1 = a;
        const bool own = n.ex >= 1 && n.ex <= 64 && n.ey >= 1 && n.ey <= TY;
        a1.trace = own ? a.trace : nullptr;
        collide_react<Real, Acc, S, TRACE>(a1, n.id, q.m, Acc(q.u), Acc(q.v), h);
    } else {
        collide_react<Real, Acc, S, false>(a, n.id, q.m, Acc(q.u), Acc(q.v), h);
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 5; ++i) L.pop[(s * 5 + i) * EP + n.e] = Real(h[s][i]);
}

// Step 2 of this thread's output node of tile (bx, by) from the LDS tile:
// returns false when the thread has no fluid output node, else the node
// index and its post-collision populations in h.  The ring nodes a gather
// can reach (x - 1 for x > 0, x + 1 for x < nx - 1, y +- 1 of a fluid node)
// were all updated in step 1; ring nodes outside the lattice are never read
// (inlet and outlet rules, solid channel walls).
template <typename Real, typename Acc, int S, bool WIDE, bool TRACE>
__device__ __forceinline__ bool pair_step2(const PairLds<Real, S> &L, const AdrArgs<Real> &a,
                                           int bx, int by, size_t &id, Acc (&h)[S][5])
{
    constexpr int EY = PairTile<Real>::EY, EX = 66, TY = EY - 2, EP = PairLds<Real, S>::EP;
    constexpr bool ULDS = PairLds<Real, S>::ULDS;
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    if (w >= TY) return false;
    const int x = bx * 64 + lane, y = by * TY + w;
    if (x >= a.nx || y >= a.ny) return false;
    id = (size_t)y * a.nxp + x;
    const int e = (w + 1) * EX + lane + 1;
    const unsigned m = ULDS ? L.mask[e] : a.mask5[id];
    if (m == MASK5_SOLID) return false;
    constexpr uint32_t LB = sizeof(Real);
    const Acc inlet_e = Acc(2) * w5<Acc>(DE) * (Acc(a.cin) - Acc(a.cref));
    const auto blk_of = [&](int s) { return LdsBlock<Real>{L.pop + s * 5 * EP}; };
    pullS_at<Acc, S>(blk_of, (uint32_t)(EP * LB), (uint32_t)(EX * LB), (uint32_t)e * LB, x, a.nx, m,
                     inlet_e, h);
    Acc u, v;
    if (ULDS) {
        u = Acc(L.vel[e]);
        v = Acc(L.vel[EP + e]);
    } else {
        using Off = off_t_<WIDE>;
        constexpr Off B = sizeof(Real);
        const Off PB = (Off)a.plane * B, o = (Off)id * B;
        const PopBlock<Real, false, WIDE> vel(a.ua, 2 * PB);
        u = Acc(vel.load(o));
        v = Acc(vel.load(o + PB));
    }
    if constexpr (TRACE) {
        AdrArgs<Real> a2 = a;
        a2.trace = a.trace2;
        collide_react<Real, Acc, S, TRACE>(a2, id, m, u, v, h);
    } else {
        collide_react<Real, Acc, S, false>(a, id, m, u, v, h);
    }
    return true;
}

// Two steps per launch (temporal blocking).  A block owns 64 x (EY - 2)
// output nodes (rows aligned to 64 nodes) and the extended tile of 66 x EY
// nodes around them (a ring of one node).  Step 1 updates the extended tile
// from the lattice in HBM and keeps the result in LDS, rounded to Real
// exactly as a store to HBM would round it.  Step 2 gathers the output nodes
// from LDS, one row per wavefront, and writes them.  A ring node is computed
// by every block whose tile it borders; its source reads mostly hit the L2
// that the XCD-aware block order shares between neighbouring tiles.  The
// lattice crosses HBM once per two steps.  Tile shape, occupancy target, the
// cache hint of the step-1 loads and whether masks and velocities stay in
// LDS (step 2 then reads global memory only for reaction rates) come from
// PairTile.  NT: streaming hint on the final stores.  Callers launch
// 64 x (EY + 1) threads per block.
template <typename Real, typename Acc, int S, bool NT, bool WIDE, bool TRACE>
__device__ __forceinline__ void pair_update(const AdrArgs<Real> &a, int bx, int by)
{
    __shared__ PairLds<Real, S> L;
    const PairNode n = pair_node(a, bx, by);
    pair_step1<Real, Acc, S, WIDE, TRACE>(L, a, n, pair_pre<Real, WIDE>(a, n));
    __syncthreads();
    size_t id;
    Acc h[S][5];
    if (pair_step2<Real, Acc, S, WIDE, TRACE>(L, a, bx, by, id, h))
        store_node<Real, Acc, S, NT, WIDE>(a, id, h);
}

}  // namespace adr
}  // namespace lbf
