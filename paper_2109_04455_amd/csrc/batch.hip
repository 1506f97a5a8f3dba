// Batched Pe x Da sweep: many independent lattices (own geometry, size,
// tau_g, velocity scale and rates) advanced together.
//
// Every instance keeps the single-lattice storage layout inside one
// workspace.  A tile table lists the (instance, tile) pairs still active; one
// launch per time step (two ADR steps per launch by default) covers the
// table, one block per slot or, for one-step ADR launches, a persistent grid
// walking it (each block takes a contiguous chunk of tiles, chunks handed
// out XCD by XCD), and blocks of steps are captured once and replayed as a
// HIP graph.  The tile count lives
// in device memory, so converged instances are dropped from the table by a
// small compaction kernel without touching the captured graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "adr_device.hpp"
#include "ctx.hpp"
#include "flow_device.hpp"

namespace lbf {
namespace {

// Per-instance device descriptor: argument blocks of the single-lattice
// kernels, for parity 0 (src = lattice 0); parity 1 swaps src and dst.
template <typename Real>
struct Inst {
    AdrArgs<Real> adr;
    FlowArgs<Real> flow;
    int tiles_x, tiles_y;    // tile grid of this instance (one-step kernels)
    int ptiles_x, ptiles_y;  // tile grid of the two-step kernel
    int ftiles_y;            // tile rows of the flow (two lattice rows per thread)
    int xf;
    double cin, cref;
};

__device__ __forceinline__ void chunk_of_block(int ntiles, int &t0, int &t1)
{
    // XCD-aware: blocks on XCD j (h mod 8 == j) take consecutive chunks
    const int G = gridDim.x, h = blockIdx.x;
    const int q = G >> 3, r = G & 7, j = h & 7, k = h >> 3;
    const int b = (G >= 8) ? j * q + (j < r ? j : r) + k : h;
    t0 = (int)((long long)ntiles * b / G);
    t1 = (int)((long long)ntiles * (b + 1) / G);
}

template <typename Real>
__device__ __forceinline__ void swap_parity(AdrArgs<Real> &a, int parity)
{
    if (parity) {
        const Real *tmp = a.src;
        a.src = a.dst;
        a.dst = const_cast<Real *>(tmp);
    }
}

// A tile table entry (instance, tile x, tile y) is the same for the whole
// block: taking it into scalar registers lets the compiler read the
// instance's argument block with scalar loads, instead of holding it per lane
// in vector registers.
__device__ __forceinline__ int4 uniform_tile(const int4 *tiles, int t)
{
    int4 v = tiles[t];
    v.x = __builtin_amdgcn_readfirstlane(v.x);
    v.y = __builtin_amdgcn_readfirstlane(v.y);
    v.z = __builtin_amdgcn_readfirstlane(v.z);
    return v;
}

// PERSIST: a fixed grid walks contiguous chunks of the tile table (next tile
// prefetched, the instance's argument block reused while the instance does
// not change).  Otherwise one block per table slot; slots past the live
// count exit at once.
template <typename Real, int S, bool NT, bool PERSIST, bool WIDE>
__global__ __launch_bounds__(256) void k_batch_adr(const Inst<Real> *__restrict__ insts, const int4 *__restrict__ tiles,
                                                   const int *ntiles, int parity, int tx, int ty)
{
    const int lx = (int)threadIdx.x % tx, ly = (int)threadIdx.x / tx;
    if (!PERSIST) {
        if ((int)blockIdx.x >= *ntiles) return;
        const int4 T = uniform_tile(tiles, blockIdx.x);
        AdrArgs<Real> a = insts[T.x].adr;
        swap_parity(a, parity);
        const int x = T.y * tx + lx, y = T.z * ty + ly;
        if (x < a.nx && y < a.ny) adr::node_update<Real, double, S, false, NT, WIDE>(a, x, y);
        return;
    }
    int t0, t1;
    chunk_of_block(*ntiles, t0, t1);
    if (t0 >= t1) return;
    int4 T = uniform_tile(tiles, t0);
    int cur = T.x;
    AdrArgs<Real> a = insts[cur].adr;
    swap_parity(a, parity);
    for (int t = t0; t < t1; ++t) {
        const int4 Tn = t + 1 < t1 ? uniform_tile(tiles, t + 1) : T;
        if (T.x != cur) {
            cur = T.x;
            a = insts[cur].adr;
            swap_parity(a, parity);
        }
        const int x = T.y * tx + lx, y = T.z * ty + ly;
        if (x < a.nx && y < a.ny) adr::node_update<Real, double, S, false, NT, WIDE>(a, x, y);
        T = Tn;
    }
}

// One block per slot of the flow tile table (slots past the live count exit
// at once): a flow tile is tx x 2 ty nodes, thread row j takes lattice rows
// 2j and 2j + 1 of the tile (FP64 arithmetic, as the single-lattice flow).
// The flow never walks the table with a persistent grid: for its short
// per-tile work a walk ran about a fifth slower than one block per tile.
template <typename Real, bool WRITE_U, bool NT, bool WIDE>
__global__ __launch_bounds__(256) void k_batch_flow(const Inst<Real> *__restrict__ insts,
                                                    const int4 *__restrict__ tiles,
                                                    const int *__restrict__ ntiles, int parity,
                                                    int tx, int ty)
{
    if ((int)blockIdx.x >= *ntiles) return;
    const int4 T = uniform_tile(tiles, blockIdx.x);
    FlowArgs<Real> a = insts[T.x].flow;
    if (parity) {
        const Real *tmp = a.src;
        a.src = a.dst;
        a.dst = const_cast<Real *>(tmp);
    }
    const int x = T.y * tx + (int)threadIdx.x % tx;
    const int y = T.z * 2 * ty + 2 * ((int)threadIdx.x / tx);
    if (x < a.nx && y < a.ny) flow::node_update2<Real, double, WRITE_U, NT, WIDE>(a, x, y);
}

// Two flow steps of every active instance per launch: one block per slot of
// the two-step tile table (the flow's two-step tile has the ADR's shape),
// each block the two-step flow update of the single-lattice path.
template <typename Real, bool WRITE_U, bool NT, bool WIDE>
__global__ __launch_bounds__(64 * (flow::FlowPairTile<Real>::EY + 1))
__attribute__((amdgpu_waves_per_eu(flow::FlowPairTile<Real>::OCC)))
void k_batch_flow2(const Inst<Real> *__restrict__ insts, const int4 *__restrict__ tiles,
                   const int *__restrict__ ntiles, int parity)
{
    if ((int)blockIdx.x >= *ntiles) return;
    const int4 T = uniform_tile(tiles, blockIdx.x);
    FlowArgs<Real> a = insts[T.x].flow;
    if (parity) {
        const Real *tmp = a.src;
        a.src = a.dst;
        a.dst = const_cast<Real *>(tmp);
    }
    flow::pair_update<Real, double, WRITE_U, NT, WIDE>(a, T.y, T.z);
}

template <typename Real>
__global__ void k_build_tiles(const Inst<Real> *insts, const int *active, int n, int kind,
                              int4 *tiles, int *ntiles)
{
    __shared__ int base[1025];
    auto grid_of = [&](int i, int &gx, int &gy) {
        gx = kind == 1 ? insts[i].ptiles_x : insts[i].tiles_x;
        gy = kind == 1 ? insts[i].ptiles_y : (kind == 2 ? insts[i].ftiles_y : insts[i].tiles_y);
    };
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < n; ++i) {
            base[i] = acc;
            int gx, gy;
            grid_of(i, gx, gy);
            if (active[i]) acc += gx * gy;
        }
        base[n] = acc;
        *ntiles = acc;
    }
    __syncthreads();
    for (int i = 0; i < n; ++i) {
        if (!active[i]) continue;
        int gx, gy;
        grid_of(i, gx, gy);
        for (int k = threadIdx.x; k < gx * gy; k += blockDim.x)
            tiles[base[i] + k] = make_int4(i, k % gx, k / gx, 0);
    }
}

// Two steps of every active instance per launch: one block per slot of the
// two-step tile table (slots past the live count exit at once), each block
// the two-step tile update of the single-lattice path.
template <typename Real, int S, bool NT, bool WIDE>
__global__ __launch_bounds__(64 * (adr::PairTile<Real>::EY + 1))
__attribute__((amdgpu_waves_per_eu(adr::PairTile<Real>::OCC)))
void k_batch_adr2(const Inst<Real> *insts, const int4 *tiles, const int *ntiles, int parity)
{
    if ((int)blockIdx.x >= *ntiles) return;
    const int4 T = uniform_tile(tiles, blockIdx.x);
    AdrArgs<Real> a = insts[T.x].adr;
    swap_parity(a, parity);
    adr::pair_update<Real, double, S, NT, WIDE, false>(a, T.y, T.z);
}

// Outlet and inlet fluxes of every instance (one block per instance, the
// same sums as the single-lattice flux kernel), from lattice `prev_parity`.
template <typename Real>
__global__ __launch_bounds__(256) void k_batch_flux(const Inst<Real> *insts, int ns, int prev_parity,
                                                    double *out)
{
    __shared__ double sm[4][256];
    const Inst<Real> &I = insts[blockIdx.x];
    const Real *src = prev_parity ? I.adr.dst : I.adr.src;
    const size_t P = I.adr.plane;
    const uint8_t *mask5 = I.adr.mask5;
    double acc[4] = {0, 0, 0, 0};
    for (int y = threadIdx.x; y < I.adr.ny; y += blockDim.x) {
        const size_t a = (size_t)y * I.adr.nxp + I.xf, b = a + 1;
        if (mask5[a] != MASK5_SOLID && mask5[b] != MASK5_SOLID)
            for (int s = 0; s < ns; ++s)
                acc[s] += (double)src[(s * 5 + 1) * P + a] - (double)src[(s * 5 + 3) * P + b];
        const size_t i0 = (size_t)y * I.adr.nxp;
        if (mask5[i0] != MASK5_SOLID)
            acc[3] += 2.0 * (1.0 / 6.0) * (I.cin - I.cref) - 2.0 * (double)src[3 * P + i0];
    }
    for (int s = 0; s < 4; ++s) sm[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int s = 0; s < 4; ++s) sm[s][threadIdx.x] += sm[s][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int s = 0; s < 4; ++s) out[4 * blockIdx.x + s] = sm[s][0];
}

// max |u - u_prev| of every instance (one block per instance); u -> u_prev.
template <typename Real>
__global__ __launch_bounds__(256) void k_batch_du(const Inst<Real> *insts, const int *active,
                                                  Real *const *uprev, double *out)
{
    __shared__ double sm[256];
    const int i = blockIdx.x;
    if (!active[i]) {
        if (threadIdx.x == 0) out[i] = 0.0;
        return;
    }
    const FlowArgs<Real> &F = insts[i].flow;
    Real *up = uprev[i];
    double mx = 0.0;
    for (size_t k = threadIdx.x; k < 2 * F.plane; k += blockDim.x) {
        const size_t id = k < F.plane ? k : k - F.plane;
        if (F.mask9[id] & MASK9_SOLID) continue;
        const double a = (double)F.u[k], b = (double)up[k];
        double d = fabs(a - b);
        if (!isfinite(a)) d = INFINITY;
        mx = fmax(mx, d);
        up[k] = F.u[k];
    }
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sm[0];
}

}  // namespace
}  // namespace lbf

using namespace lbf;

struct lbf_batch_s {
    int n = 0;
    std::vector<lbf_params> p;
    std::vector<Ctx> ctx;  // per-instance layout and argument builders (no own workspace)
    std::vector<size_t> base;  // byte offset of each instance's block
    size_t off_ptiles = 0, off_nptiles = 0;  // tile table of the two-step kernel
    int max_ptiles = 0;
    bool pair = true;  // ADR steps two per launch (flags bit 8 of instance 0 clears it)
    bool flow_pair = true;  // flow steps likewise
    size_t off_inst = 0, off_tiles = 0, off_ntiles = 0, off_active = 0, off_obs = 0, off_du = 0,
           off_uprevp = 0, total = 0;
    int max_tiles = 0;
    int tx = 256, ty = 1, grid = 2048;
    bool persistent = true;
    bool nontemporal = true;
    bool wide = true;  // 64-bit population offsets in the node updates
    char *ws = nullptr;
    hipStream_t stream = nullptr, cap_stream = nullptr;
    std::string err;
    int gpar = 0, fpar = 0;
    bool geometry = false, flow_done = false;
    std::map<std::tuple<int, long, int>, hipGraphExec_t> graphs;
    std::vector<int> parity_of;  // ADR lattice holding each instance's current state
    std::vector<long> steps_of;
    // state of the current ADR run (lbf_batch_run starts it, lbf_batch_resume
    // continues it): active instances, the eps of each one's last check, its
    // last observables and step count, the steps taken by the run
    bool running = false;
    std::vector<int> act;
    std::vector<double> prev, eps, prod;
    std::vector<long> steps_i;
    long steps = 0;
    int nact = 0;
};

namespace {

lbf_status bfail(lbf_batch b, lbf_status s, const std::string &m)
{
    if (b) b->err = m;
    return s;
}

lbf_status bhip(lbf_batch b, hipError_t e, const char *what)
{
    return bfail(b, LBF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename Real>
void fill_insts(lbf_batch b, std::vector<Inst<Real>> &v)
{
    v.resize(b->n);
    for (int i = 0; i < b->n; ++i) {
        Ctx *c = &b->ctx[i];
        Inst<Real> I{};
        I.adr = adr_args<Real>(c, 0);
        I.flow = flow_args<Real>(c, 0);
        I.tiles_x = (c->p.nx + b->tx - 1) / b->tx;
        I.tiles_y = (c->p.ny + b->ty - 1) / b->ty;
        I.ftiles_y = (c->p.ny + 2 * b->ty - 1) / (2 * b->ty);
        int ptx, pty;
        pair_tile(c->p.real_bytes, ptx, pty);
        I.ptiles_x = (c->p.nx + ptx - 1) / ptx;
        I.ptiles_y = (c->p.ny + pty - 1) / pty;
        I.xf = c->xf;
        I.cin = c->p.c_in;
        I.cref = c->cref;
        v[i] = I;
    }
}

hipError_t upload_insts(lbf_batch b)
{
    if (b->p[0].real_bytes == 4) {
        std::vector<Inst<float>> v;
        fill_insts(b, v);
        hipError_t e = hipMemcpyAsync(b->ws + b->off_inst, v.data(), v.size() * sizeof(v[0]),
                                      hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        return e;
    }
    std::vector<Inst<double>> v;
    fill_insts(b, v);
    hipError_t e = hipMemcpyAsync(b->ws + b->off_inst, v.data(), v.size() * sizeof(v[0]),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
}

// Upload the active flags and rebuild the tile tables: the two-step table,
// and in the one-step slot the one-step tiles or, for the flow phase, the
// flow tiles.
hipError_t set_active(lbf_batch b, const std::vector<int> &act, bool flow = false)
{
    hipError_t e = hipMemcpyAsync(b->ws + b->off_active, act.data(), act.size() * sizeof(int),
                                  hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return e;
    for (int pair = 0; pair < 2 && e == hipSuccess; ++pair) {
        int4 *tiles = (int4 *)(b->ws + (pair ? b->off_ptiles : b->off_tiles));
        int *nt = (int *)(b->ws + (pair ? b->off_nptiles : b->off_ntiles));
        const int *act_d = (const int *)(b->ws + b->off_active);
        const int kind = pair ? 1 : (flow ? 2 : 0);
        if (b->p[0].real_bytes == 4)
            hipLaunchKernelGGL(k_build_tiles<float>, dim3(1), dim3(256), 0, b->stream,
                               (const Inst<float> *)(b->ws + b->off_inst), act_d, b->n, kind,
                               tiles, nt);
        else
            hipLaunchKernelGGL(k_build_tiles<double>, dim3(1), dim3(256), 0, b->stream,
                               (const Inst<double> *)(b->ws + b->off_inst), act_d, b->n, kind,
                               tiles, nt);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // act must outlive the copy
    return e;
}

template <typename Real, bool NT, bool WIDE>
void batch_launch(lbf_batch b, int kind, int parity, bool write_u, hipStream_t s)
{
    const int4 *tiles = (const int4 *)(b->ws + b->off_tiles);
    const int *nt = (const int *)(b->ws + b->off_ntiles);
    const dim3 blk(b->tx * b->ty);
    auto I = (const Inst<Real> *)(b->ws + b->off_inst);
    if (kind == KIND_ADR) {
        const dim3 ga(b->persistent ? b->grid : b->max_tiles);
        if (b->p[0].nspecies == 2) {
            if (b->persistent)
                hipLaunchKernelGGL((k_batch_adr<Real, 2, NT, true, WIDE>), ga, blk, 0, s, I, tiles, nt, parity, b->tx, b->ty);
            else
                hipLaunchKernelGGL((k_batch_adr<Real, 2, NT, false, WIDE>), ga, blk, 0, s, I, tiles, nt, parity, b->tx, b->ty);
        } else {
            if (b->persistent)
                hipLaunchKernelGGL((k_batch_adr<Real, 3, NT, true, WIDE>), ga, blk, 0, s, I, tiles, nt, parity, b->tx, b->ty);
            else
                hipLaunchKernelGGL((k_batch_adr<Real, 3, NT, false, WIDE>), ga, blk, 0, s, I, tiles, nt, parity, b->tx, b->ty);
        }
    } else {
        const dim3 gf(b->max_tiles);
        if (write_u)
            hipLaunchKernelGGL((k_batch_flow<Real, true, NT, WIDE>), gf, blk, 0, s, I, tiles, nt, parity, b->tx, b->ty);
        else
            hipLaunchKernelGGL((k_batch_flow<Real, false, NT, WIDE>), gf, blk, 0, s, I, tiles, nt, parity, b->tx, b->ty);
    }
}

template <typename Real, bool NT, bool WIDE>
void batch_pair_launch(lbf_batch b, int parity, hipStream_t s)
{
    const int4 *tiles = (const int4 *)(b->ws + b->off_ptiles);
    const int *nt = (const int *)(b->ws + b->off_nptiles);
    auto I = (const Inst<Real> *)(b->ws + b->off_inst);
    const dim3 g(b->max_ptiles), blk(64 * (adr::PairTile<Real>::EY + 1));
    if (b->p[0].nspecies == 2)
        hipLaunchKernelGGL((k_batch_adr2<Real, 2, NT, WIDE>), g, blk, 0, s, I, tiles, nt, parity);
    else
        hipLaunchKernelGGL((k_batch_adr2<Real, 3, NT, WIDE>), g, blk, 0, s, I, tiles, nt, parity);
}

// Two ADR steps of every active instance in one launch.
hipError_t enqueue_batch_pair(lbf_batch b, int parity, hipStream_t s)
{
    const int sel = (b->nontemporal ? 1 : 0) | (b->wide ? 2 : 0);
    auto launch = [&](auto real) {
        using Real = decltype(real);
        switch (sel) {
        case 0: batch_pair_launch<Real, false, false>(b, parity, s); break;
        case 1: batch_pair_launch<Real, true, false>(b, parity, s); break;
        case 2: batch_pair_launch<Real, false, true>(b, parity, s); break;
        default: batch_pair_launch<Real, true, true>(b, parity, s); break;
        }
    };
    if (b->p[0].real_bytes == 4)
        launch(float(0));
    else
        launch(double(0));
    return hipGetLastError();
}

hipError_t enqueue_batch_step(lbf_batch b, int kind, int parity, bool write_u, hipStream_t s);

template <typename Real, bool NT, bool WIDE>
void batch_flow_pair_launch(lbf_batch b, int parity, bool write_u, hipStream_t s)
{
    const int4 *tiles = (const int4 *)(b->ws + b->off_ptiles);
    const int *nt = (const int *)(b->ws + b->off_nptiles);
    auto I = (const Inst<Real> *)(b->ws + b->off_inst);
    const dim3 g(b->max_ptiles), blk(64 * (flow::FlowPairTile<Real>::EY + 1));
    if (write_u)
        hipLaunchKernelGGL((k_batch_flow2<Real, true, NT, WIDE>), g, blk, 0, s, I, tiles, nt, parity);
    else
        hipLaunchKernelGGL((k_batch_flow2<Real, false, NT, WIDE>), g, blk, 0, s, I, tiles, nt, parity);
}

// Two flow steps of every active instance in one launch.
hipError_t enqueue_batch_flow_pair(lbf_batch b, int parity, bool write_u, hipStream_t s)
{
    const int sel = (b->nontemporal ? 1 : 0) | (b->wide ? 2 : 0);
    auto launch = [&](auto real) {
        using Real = decltype(real);
        switch (sel) {
        case 0: batch_flow_pair_launch<Real, false, false>(b, parity, write_u, s); break;
        case 1: batch_flow_pair_launch<Real, true, false>(b, parity, write_u, s); break;
        case 2: batch_flow_pair_launch<Real, false, true>(b, parity, write_u, s); break;
        default: batch_flow_pair_launch<Real, true, true>(b, parity, write_u, s); break;
        }
    };
    if (b->p[0].real_bytes == 4)
        launch(float(0));
    else
        launch(double(0));
    return hipGetLastError();
}

// ADR blocks run like the single-lattice path: floor((n - 1) / 2) two-step
// launches, then single steps (the last step of a block is a single one).
// Flow blocks: floor(n / 2) two-step launches, the last of them writing the
// velocity, and a single step for an odd n.
long batch_pairs(const lbf_batch_s *b, int kind, long n)
{
    if (kind == KIND_FLOW) return b->flow_pair ? n / 2 : 0;
    return kind == KIND_ADR && b->pair && n >= 3 ? (n - 1) / 2 : 0;
}

hipError_t enqueue_batch_block(lbf_batch b, int kind, int &par, long n, hipStream_t s)
{
    const long pairs = batch_pairs(b, kind, n);
    hipError_t e = hipSuccess;
    for (long i = 0; i < pairs && e == hipSuccess; ++i, par ^= 1)
        e = kind == KIND_FLOW ? enqueue_batch_flow_pair(b, par, 2 * (i + 1) == n, s)
                              : enqueue_batch_pair(b, par, s);
    for (long i = 2 * pairs; i < n && e == hipSuccess; ++i, par ^= 1)
        e = enqueue_batch_step(b, kind, par, i == n - 1, s);
    return e;
}

hipError_t enqueue_batch_step(lbf_batch b, int kind, int parity, bool write_u, hipStream_t s)
{
    const int sel = (b->nontemporal ? 1 : 0) | (b->wide ? 2 : 0);
    auto launch = [&](auto real) {
        using Real = decltype(real);
        switch (sel) {
        case 0: batch_launch<Real, false, false>(b, kind, parity, write_u, s); break;
        case 1: batch_launch<Real, true, false>(b, kind, parity, write_u, s); break;
        case 2: batch_launch<Real, false, true>(b, kind, parity, write_u, s); break;
        default: batch_launch<Real, true, true>(b, kind, parity, write_u, s); break;
        }
    };
    if (b->p[0].real_bytes == 4)
        launch(float(0));
    else
        launch(double(0));
    return hipGetLastError();
}

// n steps of every active instance (graph replay for long blocks)
lbf_status batch_steps(lbf_batch b, int kind, long n)
{
    int &par = kind == KIND_ADR ? b->gpar : b->fpar;
    if (n < GRAPH_MIN_STEPS) {
        hipError_t e = enqueue_batch_block(b, kind, par, n, b->stream);
        if (e != hipSuccess) return bhip(b, e, "batched step");
        return LBF_OK;
    }
    const auto key = std::make_tuple(kind, n, par);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return bhip(b, e, "hipStreamBeginCapture");
        int p = par;
        const hipError_t le = enqueue_batch_block(b, kind, p, n, b->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap_stream, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bhip(b, le, "batched step during capture");
        }
        if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return bhip(b, e, "hipGraphInstantiate");
        it = b->graphs.emplace(key, ex).first;
    }
    hipError_t e = hipGraphLaunch(it->second, b->stream);
    if (e != hipSuccess) return bhip(b, e, "hipGraphLaunch");
    if ((n - batch_pairs(b, kind, n)) & 1) par ^= 1;
    return LBF_OK;
}

lbf_status batch_fluxes(lbf_batch b, std::vector<double> &o)
{
    o.assign(4 * (size_t)b->n, 0.0);
    const int prev = b->gpar ^ 1;
    if (b->p[0].real_bytes == 4)
        hipLaunchKernelGGL(k_batch_flux<float>, dim3(b->n), dim3(256), 0, b->stream,
                           (const Inst<float> *)(b->ws + b->off_inst), b->p[0].nspecies, prev,
                           (double *)(b->ws + b->off_obs));
    else
        hipLaunchKernelGGL(k_batch_flux<double>, dim3(b->n), dim3(256), 0, b->stream,
                           (const Inst<double> *)(b->ws + b->off_inst), b->p[0].nspecies, prev,
                           (double *)(b->ws + b->off_obs));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(o.data(), b->ws + b->off_obs, o.size() * sizeof(double),
                           hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "batched flux");
    return LBF_OK;
}

}  // namespace

extern "C" {

lbf_status lbf_batch_create(int n, const lbf_params *params, lbf_batch *out)
{
    if (!out) return LBF_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 1024 || !params) return LBF_EINVAL;
    lbf_batch b = new (std::nothrow) lbf_batch_s();
    if (!b) return LBF_ENOMEM;
    *out = b;
    b->n = n;
    b->p.assign(params, params + n);
    b->ctx.resize(n);
    const lbf_params &p0 = params[0];
    for (int i = 0; i < n; ++i) {
        std::string why;
        const lbf_params &pi = params[i];
        lbf_status st = validate_params(&pi, why);
        if (st != LBF_OK) return bfail(b, st, "instance " + std::to_string(i) + ": " + why);
        if (pi.reaction_mode != 0 || pi.boundary != 0)
            return bfail(b, LBF_EINVAL, "the batch runs link reactions in channels only");
        if (pi.real_bytes != p0.real_bytes || pi.nspecies != p0.nspecies || pi.tau_f != p0.tau_f ||
            pi.u0 != p0.u0 || pi.c_in != p0.c_in || pi.reaction_mode != p0.reaction_mode)
            return bfail(b, LBF_EINVAL, "instances must share real_bytes, nspecies, tau_f, u0, c_in");
        Ctx &c = b->ctx[i];
        c.p = pi;
        c.xf = pi.flux_col == -1 ? pi.nx - 3 : pi.flux_col;
        c.cref = storage_shift(pi);
        c.L = make_launch(pi.nx, pi.ny, pi.tile_x, pi.tile_y);
        layout(&c);
        c.valid = true;
    }
    b->tx = p0.tile_x > 0 ? p0.tile_x : 256;
    b->ty = p0.tile_y > 0 ? p0.tile_y : 1;
    b->persistent = !(p0.flags & 8);
    // streaming accesses once the instances' ADR lattices outgrow the cache
    size_t adr_state = 0;
    for (int i = 0; i < n; ++i)
        adr_state += 2 * (size_t)p0.nspecies * 5 * p0.real_bytes * b->ctx[i].plane;
    b->nontemporal = (adr_state > NT_MIN_BYTES || (p0.flags & 64)) && !(p0.flags & 2);
    b->wide = false;
    for (int i = 0; i < n; ++i)
        b->wide = b->wide || wide_lattice(b->ctx[i].plane, p0.real_bytes, params[i].flags);
    if (b->tx * b->ty > 256 || (b->tx * b->ty) % 64)
        return bfail(b, LBF_EINVAL, "batched tiles: tile_x * tile_y must be a multiple of 64, <= 256");
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    b->base.resize(n);
    int tiles = 0;
    for (int i = 0; i < n; ++i) {
        b->base[i] = take(b->ctx[i].ws_need);
        tiles += ((params[i].nx + b->tx - 1) / b->tx) * ((params[i].ny + b->ty - 1) / b->ty);
    }
    b->max_tiles = tiles;
    int ptx, pty, ptiles = 0;
    pair_tile(p0.real_bytes, ptx, pty);
    for (int i = 0; i < n; ++i)
        ptiles += ((params[i].nx + ptx - 1) / ptx) * ((params[i].ny + pty - 1) / pty);
    b->max_ptiles = ptiles;
    b->pair = !(p0.flags & 256);
    b->flow_pair = !(p0.flags & 256) && ptx == 64 &&
                   pty == (p0.real_bytes == 4 ? flow::FlowPairTile<float>::TY
                                              : flow::FlowPairTile<double>::TY);
    const size_t inst_bytes = p0.real_bytes == 4 ? sizeof(Inst<float>) : sizeof(Inst<double>);
    b->off_inst = take((size_t)n * inst_bytes);
    b->off_tiles = take((size_t)tiles * sizeof(int4));
    b->off_ntiles = take(sizeof(int));
    b->off_ptiles = take((size_t)ptiles * sizeof(int4));
    b->off_nptiles = take(sizeof(int));
    b->off_active = take((size_t)n * sizeof(int));
    b->off_obs = take((size_t)n * 4 * sizeof(double));
    b->off_du = take((size_t)n * sizeof(double));
    b->off_uprevp = take((size_t)n * sizeof(void *));
    b->total = off;
    b->parity_of.assign(n, 0);
    b->steps_of.assign(n, 0);
    return LBF_OK;
}

lbf_status lbf_batch_workspace_bytes(lbf_batch b, size_t *bytes)
{
    if (!b || !bytes || b->total == 0) return LBF_EINVAL;
    *bytes = b->total;
    return LBF_OK;
}

lbf_status lbf_batch_bind(lbf_batch b, void *ws, size_t bytes, void *stream)
{
    if (!b || b->total == 0) return LBF_EINVAL;
    if (!ws || (uintptr_t)ws % 256) return bfail(b, LBF_EINVAL, "workspace NULL or not 256-byte aligned");
    if (bytes < b->total) return bfail(b, LBF_ENOMEM, "workspace smaller than lbf_batch_workspace_bytes");
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    if (!b->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bhip(b, e, "hipStreamCreate");
    }
    b->ws = (char *)ws;
    b->stream = (hipStream_t)stream;
    for (int i = 0; i < b->n; ++i) {
        b->ctx[i].ws = b->ws + b->base[i];
        b->ctx[i].ws_bytes = b->ctx[i].ws_need;
        b->ctx[i].stream = b->stream;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        b->grid = cus * 8;
    hipError_t e = upload_insts(b);
    if (e != hipSuccess) return bhip(b, e, "upload instance table");
    std::vector<void *> up(b->n);
    for (int i = 0; i < b->n; ++i) up[i] = b->ctx[i].ptr(b->ctx[i].off.uprev);
    e = hipMemcpyAsync(b->ws + b->off_uprevp, up.data(), up.size() * sizeof(void *),
                       hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "upload pointers");
    b->geometry = b->flow_done = false;
    return LBF_OK;
}

lbf_status lbf_batch_set_geometry(lbf_batch b, const uint8_t *type_cat, const double *k_cat)
{
    if (!b || !b->ws) return bfail(b, LBF_ESTATE, "no workspace bound");
    if (!type_cat || !k_cat) return bfail(b, LBF_EINVAL, "NULL input");
    size_t off = 0;
    for (int i = 0; i < b->n; ++i) {
        Ctx *c = &b->ctx[i];
        lbf_status st = lbf_set_geometry(c, type_cat + off);
        if (st == LBF_OK) st = lbf_set_rates(c, k_cat + off);
        if (st != LBF_OK) return bfail(b, st, "instance " + std::to_string(i) + ": " + c->err);
        off += (size_t)c->p.nx * c->p.ny;
    }
    b->geometry = true;
    b->running = false;
    return LBF_OK;
}

lbf_status lbf_batch_flow(lbf_batch b, long max_steps, int check_every, double tol)
{
    if (!b || !b->ws || !b->geometry) return bfail(b, LBF_ESTATE, "geometry not set");
    if (check_every < 1 || max_steps < 0) return bfail(b, LBF_EINVAL, "bad step counts");
    b->running = false;
    for (int i = 0; i < b->n; ++i) {
        Ctx *c = &b->ctx[i];
        hipError_t e = launch_flow_init(c->p.real_bytes, flow_args<float>(c, 1), flow_args<double>(c, 1),
                                        b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ptr(c->off.uprev), c->ptr(c->off.u), 2 * c->plane * c->p.real_bytes,
                               hipMemcpyDeviceToDevice, b->stream);
        if (e != hipSuccess) return bhip(b, e, "flow init");
    }
    b->fpar = 0;
    std::vector<int> act(b->n, 1);
    hipError_t e = set_active(b, act, true);
    if (e != hipSuccess) return bhip(b, e, "tile table");
    long steps = 0;
    int nact = b->n;
    std::vector<double> du(b->n);
    while (steps < max_steps && nact > 0) {
        const long n = std::min<long>(check_every, max_steps - steps);
        for (long left = n; left > 0;) {
            const long m = std::min<long>(left, 1000);
            lbf_status st = batch_steps(b, KIND_FLOW, m);
            if (st != LBF_OK) return st;
            left -= m;
        }
        steps += n;
        if (tol > 0) {
            if (b->p[0].real_bytes == 4)
                hipLaunchKernelGGL(k_batch_du<float>, dim3(b->n), dim3(256), 0, b->stream,
                                   (const Inst<float> *)(b->ws + b->off_inst), (const int *)(b->ws + b->off_active),
                                   (float *const *)(b->ws + b->off_uprevp), (double *)(b->ws + b->off_du));
            else
                hipLaunchKernelGGL(k_batch_du<double>, dim3(b->n), dim3(256), 0, b->stream,
                                   (const Inst<double> *)(b->ws + b->off_inst), (const int *)(b->ws + b->off_active),
                                   (double *const *)(b->ws + b->off_uprevp), (double *)(b->ws + b->off_du));
            e = hipGetLastError();
            if (e == hipSuccess)
                e = hipMemcpyAsync(du.data(), b->ws + b->off_du, du.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, b->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
            if (e != hipSuccess) return bhip(b, e, "flow residual");
            bool changed = false;
            for (int i = 0; i < b->n; ++i) {
                if (!act[i]) continue;
                if (!std::isfinite(du[i])) return bfail(b, LBF_EDIVERGED, "non-finite flow velocity");
                if (n == check_every && du[i] <= tol * std::fabs(b->p[i].u0)) {
                    act[i] = 0;
                    --nact;
                    changed = true;
                }
            }
            if (changed) {
                e = set_active(b, act, true);
                if (e != hipSuccess) return bhip(b, e, "tile table");
            }
        }
    }
    // every instance's velocity is in its own u buffer (written by the last
    // step of each block); all instances used the same flow parity sequence
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "flow");
    for (int i = 0; i < b->n; ++i) {
        b->ctx[i].velocity_set = true;
        b->ctx[i].flow_ready = true;
    }
    b->flow_done = true;
    return LBF_OK;
}

namespace {

// Advance the current run by `more` steps (checks every check_every steps
// counted from the start of the run), dropping instances whose check is
// steady; then hand each instance's state and observables out.
lbf_status batch_advance(lbf_batch b, long more, int check_every, double tol, double *eps_host,
                         double *prod_host, long *steps_host)
{
    const int ns = b->p[0].nspecies;
    const long end = b->steps + more;
    std::vector<double> o;
    while (b->steps < end && b->nact > 0) {
        const long n = std::min<long>(check_every - b->steps % check_every, end - b->steps);
        for (long left = n; left > 0;) {
            const long m = std::min<long>(left, 1000);
            lbf_status st = batch_steps(b, KIND_ADR, m);
            if (st != LBF_OK) return st;
            left -= m;
        }
        b->steps += n;
        const bool last = b->steps >= end;
        const bool check = b->steps % check_every == 0;
        if ((tol > 0 && check) || last) {
            lbf_status st = batch_fluxes(b, o);
            if (st != LBF_OK) return st;
            bool changed = false;
            for (int i = 0; i < b->n; ++i) {
                if (!b->act[i]) continue;
                double tot = 0;
                for (int s = 0; s < ns; ++s) tot += o[4 * i + s];
                if (!std::isfinite(tot)) return bfail(b, LBF_EDIVERGED, "non-finite flux");
                const double e_i = tot != 0 ? o[4 * i + ns - 1] / tot : NAN;
                b->eps[i] = e_i;
                b->prod[i] = o[4 * i + ns - 1];
                b->steps_i[i] = b->steps;
                b->parity_of[i] = b->gpar;
                if (!check) continue;  // a call ending between checks only observes
                const bool conv = tol > 0 && steady_check(&o[4 * i], ns, o[4 * i + 3], e_i,
                                                          b->prev[i], tol);
                b->prev[i] = e_i;
                if (conv) {
                    b->act[i] = 0;
                    --b->nact;
                    changed = true;
                }
            }
            if (changed && b->nact > 0) {
                hipError_t e = set_active(b, b->act);
                if (e != hipSuccess) return bhip(b, e, "tile table");
            }
        }
    }
    for (int i = 0; i < b->n; ++i) {
        b->ctx[i].gpar = b->parity_of[i];
        b->ctx[i].adr_steps = b->steps_i[i];
        b->steps_of[i] = b->steps_i[i];
        if (eps_host) eps_host[i] = b->eps[i];
        if (prod_host) prod_host[i] = b->prod[i];
        if (steps_host) steps_host[i] = b->steps_i[i];
    }
    if (tol > 0 && b->nact > 0) return bfail(b, LBF_ENOTCONV, "some instances did not converge");
    return LBF_OK;
}

}  // namespace

lbf_status lbf_batch_run(lbf_batch b, long max_steps, int check_every, double tol, double *eps_host,
                         double *prod_host, long *steps_host)
{
    if (!b || !b->ws || !b->flow_done) return bfail(b, LBF_ESTATE, "run lbf_batch_flow first");
    if (check_every < 1 || max_steps < 1) return bfail(b, LBF_EINVAL, "bad step counts");
    const int ns = b->p[0].nspecies;
    b->running = false;
    for (int i = 0; i < b->n; ++i) {
        Ctx *c = &b->ctx[i];
        hipError_t e = launch_velocity_handoff(c->p.real_bytes, c->ptr(c->off.u), c->ptr(c->off.ua),
                                               (const uint8_t *)c->ptr(c->off.mask5), c->p.vel_scale,
                                               c->plane, b->stream);
        if (e == hipSuccess)
            e = launch_adr_init(c->p.real_bytes, ns, adr_args<float>(c, 1), adr_args<double>(c, 1),
                                b->stream);
        if (e != hipSuccess) return bhip(b, e, "ADR init");
        c->adr_ready = true;
        c->gpar = 0;
    }
    b->gpar = 0;
    b->act.assign(b->n, 1);
    hipError_t e = set_active(b, b->act);
    if (e != hipSuccess) return bhip(b, e, "tile table");
    b->prev.assign(b->n, NAN);
    b->eps.assign(b->n, NAN);
    b->prod.assign(b->n, 0.0);
    b->steps_i.assign(b->n, 0);
    b->steps = 0;
    b->nact = b->n;
    b->running = true;
    return batch_advance(b, max_steps, check_every, tol, eps_host, prod_host, steps_host);
}

lbf_status lbf_batch_resume(lbf_batch b, long more_steps, int check_every, double tol,
                            double *eps_host, double *prod_host, long *steps_host)
{
    if (!b || !b->ws || !b->running) return bfail(b, LBF_ESTATE, "no run to resume (lbf_batch_run first)");
    if (check_every < 1 || more_steps < 1) return bfail(b, LBF_EINVAL, "bad step counts");
    return batch_advance(b, more_steps, check_every, tol, eps_host, prod_host, steps_host);
}

lbf_status lbf_batch_get_concentration(lbf_batch b, int i, int species, void *out)
{
    if (!b || i < 0 || i >= b->n) return LBF_EINVAL;
    lbf_status st = lbf_get_concentration(&b->ctx[i], species, out);
    if (st != LBF_OK) return bfail(b, st, b->ctx[i].err);
    return LBF_OK;
}

lbf_status lbf_batch_time_steps(lbf_batch b, long nsteps, double *ms)
{
    if (!b || !b->ws || !b->flow_done) return bfail(b, LBF_ESTATE, "run lbf_batch_flow first");
    b->running = false;  // steps every instance outside a run's bookkeeping
    std::vector<int> act(b->n, 1);
    hipError_t e = set_active(b, act);
    if (e != hipSuccess) return bhip(b, e, "tile table");
    hipEvent_t a = nullptr, z = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&z);
    if (e != hipSuccess) return bhip(b, e, "hipEventCreate");
    lbf_status st = LBF_OK;
    e = hipEventRecord(a, b->stream);
    for (long done = 0; e == hipSuccess && st == LBF_OK && done < nsteps;) {
        const long m = std::min<long>(1000, nsteps - done);
        st = batch_steps(b, KIND_ADR, m);
        done += m;
    }
    if (e == hipSuccess) e = hipEventRecord(z, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(z);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, z);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
    if (st != LBF_OK) return st;
    if (e != hipSuccess) return bhip(b, e, "timing");
    if (ms) *ms = t;
    return LBF_OK;
}

const char *lbf_batch_last_error(lbf_batch b) { return b ? b->err.c_str() : "NULL batch"; }

void lbf_batch_destroy(lbf_batch b)
{
    if (!b) return;
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

}  // extern "C"
