// Reverse-mode (adjoint) gradient of the efficiency with respect to the
// per-node rate k, for catalyst-placement studies.
//
// For a frozen velocity field the ADR step is an affine map of the
// populations.  With g(m) the pre-collision populations and
// z(m) = R(Col(g(m))) the post-collision ones (R: the link reactions of
// Eq. source_lbm, Col: the BGK collision), g(m+1) = Str z(m) + b (Str: pull
// streaming with the bounce-back / anti-bounce-back rules of Eq. BC).  The
// objective eps = f(N) depends on z(M-1) through the outlet fluxes N.
// Adjoint variables nu(m) = d eps / d g(m) obey
//     lambda(m) = Str^T nu(m+1)         (gather from the downstream nodes)
//     nu(m)     = (R Col)^T lambda(m)   (local, per node)
// and the gradient collects, for every link (x, i) into a catalytic node
// sigma = x + c_i with reaction src -> prod,
//     d eps / d k(sigma) += w_i C_src(x, m) [lambda_prod,i(x,m) - lambda_src,i(x,m)].
// The transpose needs no forward state except C_src at the fluid nodes next
// to catalysts (the "trace"), which the forward (or a recomputation from
// checkpoints) records.
#include <algorithm>
#include <cmath>
#include <vector>

#include "adr_device.hpp"
#include "gather_src.hpp"
#include "ctx.hpp"
#include "stencil.hpp"

namespace lbf {
namespace {

enum { DE = 1, DN = 2, DW = 3, DS = 4 };

template <typename Real>
__device__ __forceinline__ Real w5(int i)
{
    return i == 0 ? Real(1) / Real(3) : Real(1) / Real(6);
}

template <typename Real>
struct AdjArgs {
    const Real *nu_src;   // nu(m+1) [S][5][plane]
    Real *nu_dst;         // nu(m)
    const Real *ua;
    const uint8_t *mask5;
    const uint8_t *type;
    const Real *kr;
    const int32_t *trace_idx;
    const Real *trace;    // (C_A, C_B) of step m at the trace nodes
    const Real *trace2;   // two-step launches: the same for step m - 1
    double *acc;          // [ntrace][4] per-link gradient accumulators
    int nx, ny, nxp;
    size_t plane;
    double omega;
    Launch L;
};

// The gather of one adjoint step at node x: lam(m) from nu(m+1).  blk_of(s)
// addresses species s's 5 planes with byte offsets: PB between planes, RB
// between rows, o the node's own.  Sources are chosen by offset and all
// loads are issued before any arithmetic (no wait per direction).
template <typename Real, int S, typename BlkOf, typename Off>
__device__ __forceinline__ void adj_gather(const BlkOf &blk_of, Off PB, Off RB, Off o, int x,
                                           int nx, unsigned m, Real (&lam)[S][5])
{
    constexpr Off B = sizeof(Real);
    const bool in = x == 0, out = x == nx - 1;
    // z_E(x) feeds g_E(x+1), or g_W(x) by bounce-back, or the outlet rule;
    // z_W(x) feeds g_W(x-1), or g_E(x) by bounce-back / the inlet rule
    Off src[5];
    gather::adj_sources<Off>(B, PB, RB, o, x, nx, m, src);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const auto nu = blk_of(s);
#pragma unroll
        for (int i = 0; i < 5; ++i) lam[s][i] = nu.load(src[i]);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (in && s == 0) lam[s][DW] = -lam[s][DW];
        if (out) {
            // lam[s][DE] holds nu_W(x) here.  Outlet: every post-collision
            // population enters C_b of g_W
            const Real nw = lam[s][DE];
            lam[s][DE] = -nw;
            const Real ow = Real(2) * w5<Real>(DW) * nw;
#pragma unroll
            for (int i = 0; i < 5; ++i) lam[s][i] += ow;
        }
    }
}

// The local part of one adjoint step at fluid node id: the gradient terms of
// its catalytic links (added to the accumulators when `own`), then
// nu(m) = (R Col)^T lam into out.  trace: (C_A, C_B) of step m.  The node
// arithmetic is FP64 whatever the storage type, as in the forward collision.
template <typename Real, int S>
__device__ __forceinline__ void adj_local(const AdjArgs<Real> &a, const Real *trace, size_t id,
                                          unsigned m, Real u_, Real v_, bool own,
                                          const Real (&lam_)[S][5], Real (&out)[S][5])
{
    // lam is widened to FP64 at each use (exact), not held widened: 15
    // storage-width registers instead of 30 while the link loads travel
    const auto lam = [&](int s, int i) { return (double)lam_[s][i]; };
    double rsrc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) rsrc[s] = 0;
    if (m & 0xF0u) {
        const int off[5] = {0, 1, a.nxp, -1, -a.nxp};
        const int t = a.trace_idx[id];
        // everything the links need is loaded before any use: rate and type
        // of the four neighbours (index clamped into the plane), the trace,
        // and for the owning block the node's four link accumulators (a
        // load issued only after a link's term is known would put its
        // latency on every catalytic-adjacent node's path)
        Real kv[5];
        uint8_t tv[5];
#pragma unroll
        for (int i = 1; i < 5; ++i) {
            const long j = (long)id + off[i];
            const size_t sid = (size_t)(j < 0 ? 0 : (j >= (long)a.plane ? (long)a.plane - 1 : j));
            kv[i] = a.kr[sid];
            tv[i] = a.type[sid];
        }
        const double ca = (double)trace[2 * t], cb = (double)trace[2 * t + 1];
        double *acc = a.acc + 4 * (size_t)t;
        double ac[4] = {0, 0, 0, 0};
        if (own) {
#pragma unroll
            for (int i = 0; i < 4; ++i) ac[i] = acc[i];
        }
#pragma unroll
        for (int i = 1; i < 5; ++i) {
            if (!((m >> (3 + i)) & 1u)) continue;
            const double kap = (double)kv[i] * w5<double>(i);
            double g;
            if (tv[i] == 2) {
                const double d = lam(1, i) - lam(0, i);
                g = w5<double>(i) * ca * d;
                rsrc[0] += kap * d;
            } else {
                const double d = lam(S - 1, i) - lam(1, i);
                g = w5<double>(i) * cb * d;
                rsrc[1] += kap * d;
            }
            ac[i - 1] += g;
        }
        // the node's accumulators have one owner: links without a reaction
        // write back their unchanged value
        if (own) {
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = ac[i];
        }
    }
    // (R Col)^T: nu_j = (1 - omega) lam_j + omega sum_i e_i lam_i + rsrc
    const double u = (double)u_, v = (double)v_, uu = 1.5 * (u * u + v * v);
    double e[5];
    e[0] = w5<double>(0) * (1.0 - uu);
    e[DE] = w5<double>(DE) * (1.0 + 3.0 * u + 4.5 * u * u - uu);
    e[DN] = w5<double>(DN) * (1.0 + 3.0 * v + 4.5 * v * v - uu);
    e[DW] = w5<double>(DW) * (1.0 - 3.0 * u + 4.5 * u * u - uu);
    e[DS] = w5<double>(DS) * (1.0 - 3.0 * v + 4.5 * v * v - uu);
    const double keep = 1.0 - a.omega;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const double M = e[0] * lam(s, 0) + e[1] * lam(s, 1) + e[2] * lam(s, 2) +
                         e[3] * lam(s, 3) + e[4] * lam(s, 4);
        const double add = a.omega * M + rsrc[s];
#pragma unroll
        for (int i = 0; i < 5; ++i) out[s][i] = Real(keep * lam(s, i) + add);
    }
}

// One adjoint step at node x for all species.
template <typename Real, int S, bool NT, bool WIDE>
__global__ __launch_bounds__(1024) void k_adjoint_step(AdjArgs<Real> a)
{
    int x, y;
    tile_coords(a.L, x, y);
    if (x >= a.nx || y >= a.ny) return;
    const size_t id = (size_t)y * a.nxp + x;
    const unsigned m = a.mask5[id];
    if (m == MASK5_SOLID) return;
    const size_t P = a.plane;
    // byte offsets from each species' block, as in the forward gather
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    const Off PB = (Off)P * B, RB = (Off)a.nxp * B, o = (Off)id * B;
    const auto nu = [&](int s) { return PopBlock<Real, NT, WIDE>(a.nu_src + (size_t)s * 5 * P, 5 * PB); };
    Real lam[S][5];
    adj_gather<Real, S>(nu, PB, RB, o, x, a.nx, m, lam);
    const PopBlock<Real, false, WIDE> vel(a.ua, 2 * PB);
    Real out[S][5];
    adj_local<Real, S>(a, a.trace, id, m, vel.load(o), vel.load(o + PB), true, lam, out);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const PopBlock<Real, NT, WIDE> dst(a.nu_dst + (size_t)s * 5 * P, 5 * PB);
#pragma unroll
        for (int i = 0; i < 5; ++i) dst.store(o + i * PB, out[s][i]);
    }
}

// Two adjoint steps per launch (m, then m - 1), the tiling of the forward
// two-step launch: step m updates the extended tile (output nodes and a
// one-node ring) from nu(m+1) in HBM into LDS; step m - 1 gathers the output
// nodes from LDS and writes nu(m-1).  Gradient terms are added by the block
// owning the node only (ring nodes are computed by every block they border),
// in the order of two single steps.  Masks and velocities stay in LDS with
// FP32 state, as in the forward.
template <typename Real, int S, bool NT, bool WIDE>
__global__ __launch_bounds__(64 * (adr::PairTile<Real>::EY + 1))
__attribute__((amdgpu_waves_per_eu(adr::PairTile<Real>::OCC))) void k_adjoint_step2(AdjArgs<Real> a)
{
    constexpr int EY = adr::PairTile<Real>::EY, EX = 66, TY = EY - 2, EP = EX * EY;
    constexpr bool ULDS = adr::PairTile<Real>::ULDS;
    __shared__ Real lds[5 * S * EP];
    __shared__ Real lvel[ULDS ? 2 * EP : 1];
    __shared__ uint8_t lmask[ULDS ? EP : 1];
    using Off = off_t_<WIDE>;
    constexpr Off B = sizeof(Real);
    int bx, by;
    tile_of_block(a.L, bx, by);
    const int x0 = bx * 64, y0 = by * TY;  // first output node
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    const size_t P = a.plane;
    const Off PB = (Off)P * B;
    {
        const bool ring = w >= EY;
        const int ex = ring ? ((lane & 1) ? EX - 1 : 0) : lane + 1, ey = ring ? lane >> 1 : w;
        const int x = x0 - 1 + ex, y = y0 - 1 + ey;
        if (ey < EY && x >= 0 && x < a.nx && y >= 0 && y < a.ny) {
            const size_t id = (size_t)y * a.nxp + x;
            const int e = ey * EX + ex;
            const unsigned m = a.mask5[id];
            if (ULDS) lmask[e] = (uint8_t)m;
            if (m != MASK5_SOLID) {
                const Off o = (Off)id * B;
                const auto nu = [&](int s) {
                    return PopBlock<Real, false, WIDE>(a.nu_src + (size_t)s * 5 * P, 5 * PB);
                };
                Real lam[S][5];
                adj_gather<Real, S>(nu, PB, (Off)a.nxp * B, o, x, a.nx, m, lam);
                const PopBlock<Real, false, WIDE> vel(a.ua, 2 * PB);
                const Real u = vel.load(o), v = vel.load(o + PB);
                if (ULDS) {
                    lvel[e] = u;
                    lvel[EP + e] = v;
                }
                const bool own = ex >= 1 && ex <= 64 && ey >= 1 && ey <= TY;
                Real out[S][5];
                adj_local<Real, S>(a, a.trace, id, m, u, v, own, lam, out);
#pragma unroll
                for (int s = 0; s < S; ++s)
#pragma unroll
                    for (int i = 0; i < 5; ++i) lds[(s * 5 + i) * EP + e] = out[s][i];
            }
        }
    }
    __syncthreads();
    // Step m - 1 on the output rows.  The ring nodes a gather can reach
    // (x - 1 for x > 0, x + 1 for x < nx - 1, y +- 1 of a fluid node) were
    // all updated above.
    if (w >= TY) return;
    const int x = x0 + lane, y = y0 + w;
    if (x >= a.nx || y >= a.ny) return;
    const size_t id = (size_t)y * a.nxp + x;
    const int e = (w + 1) * EX + lane + 1;
    const unsigned m = ULDS ? lmask[e] : a.mask5[id];
    if (m == MASK5_SOLID) return;
    constexpr uint32_t LB = sizeof(Real);
    const auto nu = [&](int s) { return LdsBlock<Real>{lds + s * 5 * EP}; };
    Real lam[S][5];
    adj_gather<Real, S>(nu, (uint32_t)(EP * LB), (uint32_t)(EX * LB), (uint32_t)e * LB, x, a.nx, m,
                        lam);
    const Off o = (Off)id * B;
    Real u, v;
    if (ULDS) {
        u = lvel[e];
        v = lvel[EP + e];
    } else {
        const PopBlock<Real, false, WIDE> vel(a.ua, 2 * PB);
        u = vel.load(o);
        v = vel.load(o + PB);
    }
    Real out[S][5];
    adj_local<Real, S>(a, a.trace2, id, m, u, v, true, lam, out);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const PopBlock<Real, NT, WIDE> dst(a.nu_dst + (size_t)s * 5 * P, 5 * PB);
#pragma unroll
        for (int i = 0; i < 5; ++i) dst.store(o + i * PB, out[s][i]);
    }
}

// nu(T) = d eps / d g(T): +dfdN_s on g_E(xf+1), -dfdN_s on g_W(xf), zero
// elsewhere (the whole lattice is written).
template <typename Real>
__global__ void k_adjoint_seed(Real *nu, const uint8_t *mask5, int ns, int nx, int ny, int nxp,
                               size_t plane, int xf, double d0, double d1, double d2)
{
    const size_t n = (size_t)ns * 5 * plane;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t s = i / (5 * plane), q = (i / plane) % 5, id = i % plane;
        const int x = (int)(id % nxp), y = (int)(id / nxp);
        Real v = 0;
        if (y < ny && (x == xf || x == xf + 1)) {
            const size_t a = (size_t)y * nxp + xf;
            if (mask5[a] != MASK5_SOLID && mask5[a + 1] != MASK5_SOLID) {
                const double d = s == 0 ? d0 : (s == 1 ? d1 : d2);
                if (x == xf + 1 && q == DE) v = Real(d);
                if (x == xf && q == DW) v = Real(-d);
            }
        }
        nu[i] = v;
    }
}

// max |v| over an array (per-block maxima, then one block); non-finite -> inf
template <typename Real>
__global__ __launch_bounds__(256) void k_absmax(const Real *v, size_t n, double *partial)
{
    __shared__ double sm[256];
    double mx = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double a = fabs((double)v[i]);
        mx = fmax(mx, isfinite(a) ? a : INFINITY);
    }
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ void k_fill_f64(double *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// grad(sigma) = sum of the link accumulators of the fluid neighbours whose
// link points at sigma (fixed order E, N, W, S: deterministic).
__global__ void k_gather_grad(const double *acc, const int32_t *trace_idx, const uint8_t *mask5,
                              const uint8_t *type, int ns, int nx, int ny, int nxp, double *grad)
{
    const size_t n = (size_t)nx * ny;
    const int off[5] = {0, 1, nxp, -1, -nxp};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)(i / nx);
        const size_t sid = (size_t)y * nxp + x;
        const uint8_t t = type[sid];
        double gsum = 0.0;
        if (t == 2 || (t == 3 && ns == 3)) {
            for (int d = 1; d < 5; ++d) {
                // the fluid node x = sigma - c_d points at sigma along d
                const int xx = x - (d == 1 ? 1 : d == 3 ? -1 : 0);
                const int yy = y - (d == 2 ? 1 : d == 4 ? -1 : 0);
                if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) continue;
                const size_t fid = sid - off[d];
                const uint8_t m = mask5[fid];
                if (m == MASK5_SOLID || !((m >> (3 + d)) & 1u)) continue;
                gsum += acc[4 * trace_idx[fid] + d - 1];
            }
        }
        grad[i] = gsum;
    }
}

template <typename Real>
AdjArgs<Real> adj_args(Ctx *c, const void *nu_src, void *nu_dst, const void *trace, double *acc)
{
    AdjArgs<Real> a{};
    a.nu_src = (const Real *)nu_src;
    a.nu_dst = (Real *)nu_dst;
    a.ua = (const Real *)c->ptr(c->off.ua);
    a.mask5 = (const uint8_t *)c->ptr(c->off.mask5);
    a.type = (const uint8_t *)c->ptr(c->off.type);
    a.kr = (const Real *)c->ptr(c->off.kr);
    a.trace_idx = (const int32_t *)c->ptr(c->off.trace_idx);
    a.trace = (const Real *)trace;
    a.acc = acc;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nxp = c->nxp;
    a.plane = c->plane;
    a.omega = 1.0 / c->p.tau_g;
    a.L = c->L;
    return a;
}

template <typename Real>
void adjoint_launch(Ctx *c, const AdjArgs<Real> &a, hipStream_t s)
{
    const dim3 g = c->L.grid(), b = c->L.block();
    const int sel = (c->L.nontemporal ? 1 : 0) | (c->L.wide ? 2 : 0) | (c->p.nspecies == 3 ? 4 : 0);
    switch (sel) {
    case 0: hipLaunchKernelGGL((k_adjoint_step<Real, 2, false, false>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_adjoint_step<Real, 2, true, false>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_adjoint_step<Real, 2, false, true>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_adjoint_step<Real, 2, true, true>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_adjoint_step<Real, 3, false, false>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_adjoint_step<Real, 3, true, false>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_adjoint_step<Real, 3, false, true>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_adjoint_step<Real, 3, true, true>), g, b, 0, s, a); break;
    }
}

hipError_t launch_adjoint_step(Ctx *c, const void *nu_src, void *nu_dst, const void *trace,
                               double *acc, hipStream_t s)
{
    if (c->p.real_bytes == 4)
        adjoint_launch(c, adj_args<float>(c, nu_src, nu_dst, trace, acc), s);
    else
        adjoint_launch(c, adj_args<double>(c, nu_src, nu_dst, trace, acc), s);
    return hipGetLastError();
}

template <typename Real>
void adjoint_pair_launch(Ctx *c, const AdjArgs<Real> &a, hipStream_t s)
{
    const dim3 g = c->Lp.grid(), b(64 * (adr::PairTile<Real>::EY + 1));
    const int sel = (c->Lp.nontemporal ? 1 : 0) | (c->Lp.wide ? 2 : 0) | (c->p.nspecies == 3 ? 4 : 0);
    switch (sel) {
    case 0: hipLaunchKernelGGL((k_adjoint_step2<Real, 2, false, false>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_adjoint_step2<Real, 2, true, false>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_adjoint_step2<Real, 2, false, true>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_adjoint_step2<Real, 2, true, true>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_adjoint_step2<Real, 3, false, false>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_adjoint_step2<Real, 3, true, false>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_adjoint_step2<Real, 3, false, true>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_adjoint_step2<Real, 3, true, true>), g, b, 0, s, a); break;
    }
}

// Adjoint steps m and m - 1 in one launch: nu(m+1) -> nu(m-1).
hipError_t launch_adjoint_pair(Ctx *c, const void *nu_src, void *nu_dst, const void *trace_m,
                               const void *trace_m1, double *acc, hipStream_t s)
{
    if (c->p.real_bytes == 4) {
        AdjArgs<float> a = adj_args<float>(c, nu_src, nu_dst, trace_m, acc);
        a.trace2 = (const float *)trace_m1;
        a.L = c->Lp;
        adjoint_pair_launch(c, a, s);
    } else {
        AdjArgs<double> a = adj_args<double>(c, nu_src, nu_dst, trace_m, acc);
        a.trace2 = (const double *)trace_m1;
        a.L = c->Lp;
        adjoint_pair_launch(c, a, s);
    }
    return hipGetLastError();
}

// Forward step between arbitrary lattices (used by the recomputation).
hipError_t forward_step(Ctx *c, const void *src, void *dst, void *trace, hipStream_t s)
{
    AdrArgs<float> af = adr_args<float>(c, 0);
    AdrArgs<double> ad = adr_args<double>(c, 0);
    af.src = (const float *)src;
    af.dst = (float *)dst;
    af.trace = (float *)trace;
    ad.src = (const double *)src;
    ad.dst = (double *)dst;
    ad.trace = (double *)trace;
    af.L = ad.L = c->Lv;
    return launch_adr_step(c->p.real_bytes, c->p.nspecies, trace != nullptr, af, ad, s);
}

// Two forward steps from `src` into `dst` (two-step launch), recording the
// trace of each step into its slot when given.
hipError_t forward_pair(Ctx *c, const void *src, void *dst, void *trace1, void *trace2,
                        hipStream_t s)
{
    AdrArgs<float> af = adr_args<float>(c, 0);
    AdrArgs<double> ad = adr_args<double>(c, 0);
    af.src = (const float *)src;
    af.dst = (float *)dst;
    af.trace = (float *)trace1;
    af.trace2 = (float *)trace2;
    ad.src = (const double *)src;
    ad.dst = (double *)dst;
    ad.trace = (double *)trace1;
    ad.trace2 = (double *)trace2;
    af.L = ad.L = c->Lp;
    return launch_adr_pair(c->p.real_bytes, c->p.nspecies, af, ad, s);
}

struct AdjLayout {
    size_t nu[2], rec[2], ckpt, ckpt_trace, trace, acc, partial, total;
    long nseg;
    size_t lattice, slot;
};

AdjLayout adj_layout(const Ctx *c, long T, int M, int keep)
{
    AdjLayout L{};
    const size_t R = c->p.real_bytes;
    L.lattice = (size_t)c->p.nspecies * 5 * c->plane * R;
    L.slot = (size_t)std::max(c->ntrace, 1) * 2 * R;
    L.nseg = (T + M - 1) / M;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.nu[0] = take(L.lattice);
    L.nu[1] = take(L.lattice);
    L.acc = take((size_t)std::max(c->ntrace, 1) * 4 * sizeof(double));
    L.partial = take(1025 * sizeof(double));
    if (keep) {
        L.trace = take((size_t)T * L.slot);
        L.rec[0] = L.rec[1] = L.ckpt = L.ckpt_trace = 0;
    } else {
        L.rec[0] = take(L.lattice);
        L.rec[1] = take(L.lattice);
        L.ckpt = take((size_t)L.nseg * L.lattice);
        L.ckpt_trace = take((size_t)L.nseg * L.slot);
        L.trace = take((size_t)M * L.slot);
    }
    L.total = off;
    return L;
}

}  // namespace

void adjoint_release(Ctx *) {}

}  // namespace lbf

using namespace lbf;

extern "C" {

lbf_status lbf_adjoint_workspace_bytes(lbf_ctx c, long T, int M, int keep, size_t *bytes)
{
    if (!c || !bytes) return LBF_EINVAL;
    if (!c->valid) return fail(c, LBF_EINVAL, "invalid context");
    if (c->p.reaction_mode != 0 || c->p.boundary != 0)
        return fail(c, LBF_EINVAL, "the adjoint covers link reactions in a channel only");
    if (T < 1 || M < 1) return fail(c, LBF_EINVAL, "need T >= 1 and ckpt_every >= 1");
    if (!c->geometry_set) return fail(c, LBF_ESTATE, "geometry not set");
    *bytes = adj_layout(c, T, M, keep).total;
    return LBF_OK;
}

lbf_status lbf_adr_adjoint(lbf_ctx c, long T, int M, int keep, void *ws, size_t bytes,
                           double *eps_out, double *grad)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (c->p.reaction_mode != 0 || c->p.boundary != 0)
        return fail(c, LBF_EINVAL, "the adjoint covers link reactions in a channel only");
    if (T < 1 || M < 1) return fail(c, LBF_EINVAL, "need T >= 1 and ckpt_every >= 1");
    if (!ws || !grad) return fail(c, LBF_EINVAL, "NULL workspace or gradient");
    if ((uintptr_t)ws % 256) return fail(c, LBF_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (!c->adr_ready || c->adr_steps < 1)
        return fail(c, LBF_ESTATE, "the adjoint needs at least one ADR step taken");
    const AdjLayout L = adj_layout(c, T, M, keep);
    if (bytes < L.total) return fail(c, LBF_ENOMEM, "adjoint workspace too small");
    char *W = (char *)ws;
    hipStream_t s = c->stream;
    double *acc = (double *)(W + L.acc);
    const size_t nacc = (size_t)std::max(c->ntrace, 1) * 4;
    hipLaunchKernelGGL(k_fill_f64, dim3(256), dim3(256), 0, s, acc, nacc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "fill");

    auto slot = [&](size_t base, long j) { return (void *)(W + base + (size_t)j * L.slot); };
    // The objective holds the pre-collision state fixed; the current lattice
    // is its collided form with the rates of the step that made it.  Redo
    // that collision (one step from the previous lattice) with the rates set
    // now, so that eps_out is the efficiency of these rates, consistent with
    // the gradient, also after lbf_set_rates changed them.
    e = enqueue_adr_step(c, c->gpar ^ 1, s, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "window start");
    // C at the trace nodes for the window's first step (pre-collision state
    // pulled from the lattice before the current one)
    {
        AdrArgs<float> af = adr_args<float>(c, c->gpar ^ 1);
        AdrArgs<double> ad = adr_args<double>(c, c->gpar ^ 1);
        void *s0 = keep ? slot(L.trace, 0) : slot(L.ckpt_trace, 0);
        af.trace = (float *)s0;
        ad.trace = (double *)s0;
        e = launch_trace_conc(c->p.real_bytes, c->p.nspecies, af, ad,
                              (const int32_t *)c->ptr(c->off.trace_nodes), c->ntrace, s);
        if (e != hipSuccess) return hip_fail(c, e, "trace at window start");
    }
    // ---- forward T steps (as lbf_adr_run would), recording what the reverse needs
    if (!keep) {
        e = hipMemcpyAsync(W + L.ckpt, c->ptr(c->off.g[c->gpar]), L.lattice, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(c, e, "checkpoint copy");
    }
    // the last segment's trace is recorded here directly into the segment
    // trace buffer, which the reverse sweep visits first: no recompute for it
    const long last_a0 = (L.nseg - 1) * (long)M;
    auto trace_of = [&](long m) -> void * {
        if (m >= T) return nullptr;
        if (keep) return slot(L.trace, m);
        if (m % M == 0) return slot(L.ckpt_trace, m / M);
        if (m > last_a0) return slot(L.trace, m - last_a0);
        return nullptr;
    };
    auto ckpt_after = [&](long m) { return !keep && m % M == 0 && m < T; };
    // steps run two per launch where no checkpoint falls between them; the
    // last step is a single one (the outlet fluxes read the state before it)
    for (long m = 1; m <= T;) {
        const bool two = c->pair && m + 1 < T && !ckpt_after(m);
        if (two)
            e = forward_pair(c, c->ptr(c->off.g[c->gpar]), c->ptr(c->off.g[c->gpar ^ 1]),
                             trace_of(m), trace_of(m + 1), s);
        else
            e = enqueue_adr_step(c, c->gpar, s, trace_of(m));
        if (e != hipSuccess) return hip_fail(c, e, "forward step");
        c->gpar ^= 1;
        m += two ? 2 : 1;
        if (ckpt_after(m - 1)) {
            e = hipMemcpyAsync(W + L.ckpt + (size_t)((m - 1) / M) * L.lattice,
                               c->ptr(c->off.g[c->gpar]), L.lattice, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(c, e, "checkpoint copy");
        }
    }
    c->adr_steps += T;
    double o[4];
    st = compute_fluxes(c, o);
    if (st != LBF_OK) return st;
    const int ns = c->p.nspecies;
    double tot = 0;
    for (int q = 0; q < ns; ++q) tot += o[q];
    if (tot == 0) return fail(c, LBF_ESTATE, "total outlet flux is zero: eps undefined");
    const double eps = o[ns - 1] / tot;
    double dfdn[3] = {0, 0, 0};
    for (int q = 0; q < ns; ++q) dfdn[q] = -o[ns - 1] / (tot * tot) + (q == ns - 1 ? 1.0 / tot : 0.0);

    // ---- reverse
    void *nu[2] = {W + L.nu[0], W + L.nu[1]};
    if (c->p.real_bytes == 4)
        hipLaunchKernelGGL(k_adjoint_seed<float>, dim3(2048), dim3(256), 0, s, (float *)nu[0],
                           (const uint8_t *)c->ptr(c->off.mask5), ns, c->p.nx, c->p.ny, c->nxp,
                           c->plane, c->xf, dfdn[0], dfdn[1], dfdn[2]);
    else
        hipLaunchKernelGGL(k_adjoint_seed<double>, dim3(2048), dim3(256), 0, s, (double *)nu[0],
                           (const uint8_t *)c->ptr(c->off.mask5), ns, c->p.nx, c->p.ny, c->nxp,
                           c->plane, c->xf, dfdn[0], dfdn[1], dfdn[2]);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "adjoint seed");
    int cur = 0;
    // adjoint steps run two per launch (m and m - 1) within a trace window
    if (keep) {
        for (long m = T - 1; m >= 0;) {
            const bool two = c->pair && m >= 1;
            e = two ? launch_adjoint_pair(c, nu[cur], nu[cur ^ 1], slot(L.trace, m),
                                          slot(L.trace, m - 1), acc, s)
                    : launch_adjoint_step(c, nu[cur], nu[cur ^ 1], slot(L.trace, m), acc, s);
            if (e != hipSuccess) return hip_fail(c, e, "adjoint step");
            cur ^= 1;
            m -= two ? 2 : 1;
        }
    } else {
        void *rec[2] = {W + L.rec[0], W + L.rec[1]};
        for (long j = L.nseg - 1; j >= 0; --j) {
            const long a0 = j * M, a1 = std::min<long>(T, a0 + M);
            // segment trace: slot 0 is the checkpoint's, recompute the rest
            e = hipMemcpyAsync(slot(L.trace, 0), slot(L.ckpt_trace, j), L.slot, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(c, e, "segment trace copy");
            const void *src = W + L.ckpt + (size_t)j * L.lattice;
            int r = 0;
            for (long q = 1; q < a1 - a0 && j < L.nseg - 1;) {
                const bool two = c->pair && q + 1 < a1 - a0;
                e = two ? forward_pair(c, src, rec[r], slot(L.trace, q), slot(L.trace, q + 1), s)
                        : forward_step(c, src, rec[r], slot(L.trace, q), s);
                if (e != hipSuccess) return hip_fail(c, e, "recompute step");
                src = rec[r];
                r ^= 1;
                q += two ? 2 : 1;
            }
            for (long m = a1 - 1; m >= a0;) {
                const bool two = c->pair && m - 1 >= a0;
                e = two ? launch_adjoint_pair(c, nu[cur], nu[cur ^ 1], slot(L.trace, m - a0),
                                              slot(L.trace, m - 1 - a0), acc, s)
                        : launch_adjoint_step(c, nu[cur], nu[cur ^ 1], slot(L.trace, m - a0), acc, s);
                if (e != hipSuccess) return hip_fail(c, e, "adjoint step");
                cur ^= 1;
                m -= two ? 2 : 1;
            }
        }
    }
    hipLaunchKernelGGL(k_gather_grad, dim3(2048), dim3(256), 0, s, acc,
                       (const int32_t *)c->ptr(c->off.trace_idx), (const uint8_t *)c->ptr(c->off.mask5),
                       (const uint8_t *)c->ptr(c->off.type), ns, c->p.nx, c->p.ny, c->nxp, grad);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "gradient gather");
    if (eps_out) *eps_out = eps;
    return LBF_OK;
}

lbf_status lbf_adr_adjoint_steady(lbf_ctx c, long max_iters, int check_every, double tol,
                                  void *ws, size_t bytes, double *eps_out, double *grad,
                                  long *iters_done)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (c->p.reaction_mode != 0 || c->p.boundary != 0)
        return fail(c, LBF_EINVAL, "the adjoint covers link reactions in a channel only");
    if (max_iters < 1 || check_every < 1 || !(tol > 0))
        return fail(c, LBF_EINVAL, "need max_iters >= 1, check_every >= 1, tol > 0");
    if (!ws || !grad) return fail(c, LBF_EINVAL, "NULL workspace or gradient");
    if ((uintptr_t)ws % 256) return fail(c, LBF_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (!c->adr_ready || c->adr_steps < 1)
        return fail(c, LBF_ESTATE, "the steady adjoint needs a (converged) ADR state");
    const AdjLayout L = adj_layout(c, 1, 1, 1);
    if (bytes < L.total) return fail(c, LBF_ENOMEM, "adjoint workspace too small");
    char *W = (char *)ws;
    hipStream_t s = c->stream;
    double *acc = (double *)(W + L.acc);
    hipLaunchKernelGGL(k_fill_f64, dim3(256), dim3(256), 0, s, acc,
                       (size_t)std::max(c->ntrace, 1) * 4);
    // the steady concentrations at the trace nodes (constant)
    void *tr = W + L.trace;
    {
        AdrArgs<float> af = adr_args<float>(c, c->gpar ^ 1);
        AdrArgs<double> ad = adr_args<double>(c, c->gpar ^ 1);
        af.trace = (float *)tr;
        ad.trace = (double *)tr;
        hipError_t e = launch_trace_conc(c->p.real_bytes, c->p.nspecies, af, ad,
                                         (const int32_t *)c->ptr(c->off.trace_nodes), c->ntrace, s);
        if (e != hipSuccess) return hip_fail(c, e, "steady trace");
    }
    double o[4];
    st = compute_fluxes(c, o);
    if (st != LBF_OK) return st;
    const int ns = c->p.nspecies;
    double tot = 0;
    for (int q = 0; q < ns; ++q) tot += o[q];
    if (tot == 0) return fail(c, LBF_ESTATE, "total outlet flux is zero: eps undefined");
    const double eps = o[ns - 1] / tot;
    double dfdn[3] = {0, 0, 0};
    for (int q = 0; q < ns; ++q) dfdn[q] = -o[ns - 1] / (tot * tot) + (q == ns - 1 ? 1.0 / tot : 0.0);
    void *nu[2] = {W + L.nu[0], W + L.nu[1]};
    // the steps write fluid nodes only and the norm reads every entry: start
    // the second lattice at zero (the seed writes all of the first)
    {
        hipError_t e0 = hipMemsetAsync(nu[1], 0, L.lattice, s);
        if (e0 != hipSuccess) return hip_fail(c, e0, "adjoint lattice clear");
    }
    if (c->p.real_bytes == 4)
        hipLaunchKernelGGL(k_adjoint_seed<float>, dim3(2048), dim3(256), 0, s, (float *)nu[0],
                           (const uint8_t *)c->ptr(c->off.mask5), ns, c->p.nx, c->p.ny, c->nxp,
                           c->plane, c->xf, dfdn[0], dfdn[1], dfdn[2]);
    else
        hipLaunchKernelGGL(k_adjoint_seed<double>, dim3(2048), dim3(256), 0, s, (double *)nu[0],
                           (const uint8_t *)c->ptr(c->off.mask5), ns, c->p.nx, c->p.ny, c->nxp,
                           c->plane, c->xf, dfdn[0], dfdn[1], dfdn[2]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "adjoint seed");
    const size_t nlat = (size_t)ns * 5 * c->plane;
    double *partial = (double *)(W + L.partial);
    auto absmax = [&](const void *v, double *out) -> lbf_status {
        if (c->p.real_bytes == 4)
            hipLaunchKernelGGL(k_absmax<float>, dim3(1024), dim3(256), 0, s, (const float *)v, nlat, partial);
        else
            hipLaunchKernelGGL(k_absmax<double>, dim3(1024), dim3(256), 0, s, (const double *)v, nlat, partial);
        hipError_t e2 = hipGetLastError();
        if (e2 == hipSuccess) e2 = launch_du_max_partials(partial, 1024, partial + 1024, s);
        double h = 0;
        if (e2 == hipSuccess) e2 = hipMemcpyAsync(&h, partial + 1024, sizeof h, hipMemcpyDeviceToHost, s);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        if (e2 != hipSuccess) return hip_fail(c, e2, "adjoint norm");
        *out = h;
        return LBF_OK;
    };
    double n0 = 0;
    st = absmax(nu[0], &n0);
    if (st != LBF_OK) return st;
    int cur = 0;
    long it = 0;
    bool conv = false;
    while (it < max_iters) {
        const long m = std::min<long>(check_every, max_iters - it);
        // two iterations per launch where the check interval allows
        for (long q = 0; q < m;) {
            const bool two = c->pair && q + 1 < m;
            e = two ? launch_adjoint_pair(c, nu[cur], nu[cur ^ 1], tr, tr, acc, s)
                    : launch_adjoint_step(c, nu[cur], nu[cur ^ 1], tr, acc, s);
            if (e != hipSuccess) return hip_fail(c, e, "adjoint step");
            cur ^= 1;
            q += two ? 2 : 1;
        }
        it += m;
        double nn = 0;
        st = absmax(nu[cur], &nn);
        if (st != LBF_OK) return st;
        if (!std::isfinite(nn)) return fail(c, LBF_EDIVERGED, "adjoint diverged");
        if (nn <= tol * n0) {
            conv = true;
            break;
        }
    }
    hipLaunchKernelGGL(k_gather_grad, dim3(2048), dim3(256), 0, s, acc,
                       (const int32_t *)c->ptr(c->off.trace_idx), (const uint8_t *)c->ptr(c->off.mask5),
                       (const uint8_t *)c->ptr(c->off.type), ns, c->p.nx, c->p.ny, c->nxp, grad);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "gradient gather");
    if (eps_out) *eps_out = eps;
    if (iters_done) *iters_done = it;
    if (!conv) return fail(c, LBF_ENOTCONV, "steady adjoint not converged within max_iters");
    return LBF_OK;
}

}  // extern "C"
