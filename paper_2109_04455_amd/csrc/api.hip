// Host side of the C ABI (include/lbf.h): parameter validation, workspace
// layout, HIP-graph replay of step blocks, convergence loops and
// observables.  Validation happens before any HIP call so it can be
// exercised without a GPU.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "stencil.hpp"

using namespace lbf;

namespace lbf {

lbf_status fail(Ctx *c, lbf_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

lbf_status hip_fail(Ctx *c, hipError_t e, const char *what)
{
    return fail(c, LBF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

lbf_status validate_params(const lbf_params *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return LBF_EINVAL; }
    if (p->nx < 8 || p->ny < 3) { why = "need nx >= 8 and ny >= 3"; return LBF_EINVAL; }
    if ((size_t)p->nx * (size_t)p->ny > (size_t)1 << 32) { why = "lattice too large"; return LBF_EINVAL; }
    if (p->real_bytes != 4 && p->real_bytes != 8) { why = "real_bytes must be 4 or 8"; return LBF_EINVAL; }
    if (p->nspecies != 2 && p->nspecies != 3) { why = "nspecies must be 2 or 3"; return LBF_EINVAL; }
    if (p->reaction_mode != 0 && p->reaction_mode != 1) { why = "reaction_mode must be 0 or 1"; return LBF_EINVAL; }
    if (p->boundary != 0 && p->boundary != 1) { why = "boundary must be 0 (channel) or 1 (periodic)"; return LBF_EINVAL; }
    if (!(p->tau_f > 0.5) || !std::isfinite(p->tau_f)) { why = "tau_f must be > 0.5"; return LBF_EINVAL; }
    if (!(p->tau_g > 0.5) || !std::isfinite(p->tau_g)) { why = "tau_g must be > 0.5"; return LBF_EINVAL; }
    if (!(std::fabs(p->u0) < 0.3)) { why = "|u0| must be < 0.3"; return LBF_EINVAL; }
    if (!std::isfinite(p->c_in)) { why = "c_in must be finite"; return LBF_EINVAL; }
    if (!(p->vel_scale >= 0) || !std::isfinite(p->vel_scale)) { why = "vel_scale must be >= 0"; return LBF_EINVAL; }
    if (!(std::fabs(p->vel_scale * p->u0) < 0.3)) { why = "|vel_scale * u0| must be < 0.3"; return LBF_EINVAL; }
    if (p->flux_col != -1 && (p->flux_col < 1 || p->flux_col > p->nx - 2)) {
        why = "flux_col must be -1 or in [1, nx-2]";
        return LBF_EINVAL;
    }
    if (p->variant < 0 || p->variant > 2) { why = "variant must be 0, 1 or 2"; return LBF_EINVAL; }
    if (p->real_bytes == 4 && (p->flags & 4) && (p->flags & 16)) {
        // FP32 arithmetic on species A stored unshifted loses the small
        // depletion of A to rounding (~2e-4 of the field on a 512 x 128
        // cascade after 3000 steps, over the 1e-4 accuracy bar)
        why = "flags bits 2 and 4 together (unshifted A with FP32 arithmetic) are not supported";
        return LBF_EINVAL;
    }
    const bool ext = p->reaction_mode != 0 || p->boundary != 0;
    if (ext && p->variant == 2) {
        why = "the vector kernel covers link reactions in a channel only (variant 0 or 1)";
        return LBF_EINVAL;
    }
    const bool vec = !ext && (p->variant == 2 || (p->variant == 0 && p->real_bytes == 8));
    const int tx = p->tile_x > 0 ? p->tile_x : (vec ? 64 : 256);
    const int ty = p->tile_y > 0 ? p->tile_y : (vec ? 4 : 1);
    const int maxb = vec ? 256 : 1024;
    if (p->tile_x < 0 || p->tile_y < 0 || tx * ty > maxb || (tx * ty) % 64 != 0) {
        why = "tile_x * tile_y must be a multiple of 64 and <= 1024 (<= 256 for vectors)";
        return LBF_EINVAL;
    }
    return LBF_OK;
}

// Byte layout of the workspace.  Every block is 256-byte aligned.
void layout(Ctx *c)
{
    const lbf_params &p = c->p;
    c->nxp = (int)align_up((size_t)p.nx, ROW_ALIGN);
    c->plane = (size_t)c->nxp * p.ny;
    const size_t P = c->plane, R = (size_t)p.real_bytes;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    c->off.type = take(P);
    c->off.mask5 = take(P);
    c->off.mask9 = take(2 * P);
    c->off.trace_idx = take(4 * P);
    c->off.trace_nodes = take(4 * P);
    c->off.kr = take(R * P);
    c->off.f[0] = take(9 * R * P);
    c->off.f[1] = take(9 * R * P);
    c->off.u = take(2 * R * P);
    c->off.uprev = take(2 * R * P);
    c->off.ua = take(2 * R * P);
    c->off.g[0] = take((size_t)p.nspecies * 5 * R * P);
    c->off.g[1] = take((size_t)p.nspecies * 5 * R * P);
    c->off.obs = take(16 * sizeof(double));
    c->off.partial = take(1024 * sizeof(double));
    c->off.counter = take(256);
    c->ws_need = off;
}

// Enqueue one ADR step from lattice `src_buf` (writing the other one).
hipError_t enqueue_adr_step(Ctx *c, int src_buf, hipStream_t s, void *trace_slot)
{
    AdrArgs<float> af = adr_args<float>(c, src_buf);
    AdrArgs<double> ad = adr_args<double>(c, src_buf);
    af.trace = (float *)trace_slot;
    ad.trace = (double *)trace_slot;
    af.L = ad.L = c->Lv;
    return launch_adr_step(c->p.real_bytes, c->p.nspecies, trace_slot != nullptr, af, ad, s);
}

// Enqueue two ADR steps from lattice `src_buf`; the result lands in the
// other lattice, as after one step (the intermediate state stays in LDS).
hipError_t enqueue_adr_pair(Ctx *c, int src_buf, hipStream_t s)
{
    AdrArgs<float> af = adr_args<float>(c, src_buf);
    AdrArgs<double> ad = adr_args<double>(c, src_buf);
    if (c->march) {
        af.L = c->Lm;
        return launch_adr_march(c->p.nspecies, af, s);
    }
    af.L = ad.L = c->Lp;
    return launch_adr_pair(c->p.real_bytes, c->p.nspecies, af, ad, s);
}

// An ADR block of n steps runs as `pairs` two-step launches followed by
// n - 2 pairs single steps; the last step is always a single one, so that
// the other lattice holds the state one step back (the outlet fluxes read
// it).  Returns the number of lattice swaps.
long adr_pairs(const Ctx *c, long n) { return c->pair && n >= 3 ? (n - 1) / 2 : 0; }

hipError_t enqueue_adr_block(Ctx *c, int &par, long n, hipStream_t s)
{
    const long pairs = adr_pairs(c, n);
    hipError_t e = hipSuccess;
    for (long i = 0; i < pairs && e == hipSuccess; ++i, par ^= 1) e = enqueue_adr_pair(c, par, s);
    for (long i = 2 * pairs; i < n && e == hipSuccess; ++i, par ^= 1)
        e = enqueue_adr_step(c, par, s, nullptr);
    return e;
}

hipError_t enqueue_flow_step(Ctx *c, int src_buf, bool write_u, hipStream_t s)
{
    return launch_flow_step(c->p.real_bytes, write_u, flow_args<float>(c, src_buf),
                            flow_args<double>(c, src_buf), s);
}

// Two-step launches in a flow block of n steps (each swaps the lattices once).
long flow_pairs(const Ctx *c, long n) { return c->flow_pair ? n / 2 : 0; }

// A flow block of n steps from lattice par: two steps per launch where the
// context runs them, a single step for an odd remainder; the velocity is
// written by the block's last step (its second step for a final pair).
hipError_t enqueue_flow_block(Ctx *c, int &par, long n, hipStream_t s)
{
    hipError_t e = hipSuccess;
    long i = 0;
    if (c->flow_pair) {
        for (; i + 2 <= n && e == hipSuccess; i += 2, par ^= 1) {
            FlowArgs<float> af = flow_args<float>(c, par);
            FlowArgs<double> ad = flow_args<double>(c, par);
            const bool fp32 = af.L.fp32_math;
            af.L = ad.L = c->Lfp;
            af.L.fp32_math = ad.L.fp32_math = fp32;
            e = launch_flow_pair(c->p.real_bytes, i + 2 == n, af, ad, s);
        }
    }
    for (; i < n && e == hipSuccess; ++i, par ^= 1) e = enqueue_flow_step(c, par, i == n - 1, s);
    return e;
}

// The instantiated graph of n consecutive steps starting from lattice par
// (captured and instantiated on first use).
lbf_status graph_of(Ctx *c, int kind, long n, int par, hipGraphExec_t *out)
{
    const auto key = std::make_tuple(kind, n, par);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
        int p = par;
        hipError_t le = hipSuccess;
        if (kind == KIND_ADR) {
            le = enqueue_adr_block(c, p, n, c->cap_stream);
        } else {
            le = enqueue_flow_block(c, p, n, c->cap_stream);
        }
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->cap_stream, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(c, le, "step launch during capture");
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
        it = c->graphs.emplace(key, ex).first;
    }
    *out = it->second;
    return LBF_OK;
}

// Replay (capturing on first use) a graph of n consecutive steps.
lbf_status run_steps(Ctx *c, int kind, long n)
{
    if (n <= 0) return LBF_OK;
    int &par = kind == KIND_ADR ? c->gpar : c->fpar;
    if (n < GRAPH_MIN_STEPS) {
        if (kind == KIND_ADR) {
            hipError_t e = enqueue_adr_block(c, par, n, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "step launch");
            return LBF_OK;
        }
        hipError_t e = enqueue_flow_block(c, par, n, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "step launch");
        return LBF_OK;
    }
    hipGraphExec_t ex = nullptr;
    lbf_status st = graph_of(c, kind, n, par, &ex);
    if (st != LBF_OK) return st;
    hipError_t e = hipGraphLaunch(ex, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    const long swaps = n - (kind == KIND_ADR ? adr_pairs(c, n) : flow_pairs(c, n));
    if (swaps & 1) par ^= 1;
    return LBF_OK;
}

void clear_graphs(Ctx *c)
{
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

lbf_status read_obs(Ctx *c, double *host, int n)
{
    hipError_t e = hipMemcpyAsync(host, c->ptr(c->off.obs), sizeof(double) * n,
                                  hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync(obs)");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    return LBF_OK;
}

// Fluxes of the last step into obs[0..3] (N_A, N_B, N_C, inflow_A).
lbf_status compute_fluxes(Ctx *c, double *out4)
{
    if (c->adr_steps < 1) return fail(c, LBF_ESTATE, "no ADR step taken yet");
    const int prev = c->gpar ^ 1;
    hipError_t e = launch_flux(c->p.real_bytes, c->p.nspecies, c->ptr(c->off.g[prev]),
                               (const uint8_t *)c->ptr(c->off.mask5), c->p.nx, c->p.ny, c->nxp,
                               c->plane, c->xf, c->p.c_in, c->cref, (double *)c->ptr(c->off.obs),
                               c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "flux kernel");
    double h[4];
    lbf_status st = read_obs(c, h, 4);
    if (st != LBF_OK) return st;
    std::memcpy(out4, h, sizeof h);
    for (int s = 0; s < 4; ++s)
        if (!std::isfinite(h[s])) return fail(c, LBF_EDIVERGED, "non-finite outlet flux");
    return LBF_OK;
}

double efficiency_of(const double *N, int ns)
{
    double tot = 0;
    for (int s = 0; s < ns; ++s) tot += N[s];
    return tot != 0 ? N[ns - 1] / tot : NAN;
}

lbf_status check_ready(Ctx *c, bool need_geometry)
{
    if (!c) return LBF_EINVAL;
    if (!c->ws) return fail(c, LBF_ESTATE, "no workspace bound");
    if (need_geometry && !c->geometry_set) return fail(c, LBF_ESTATE, "geometry not set");
    return LBF_OK;
}

}  // namespace lbf

extern "C" {

int lbf_version(void) { return 1; }

const char *lbf_status_str(lbf_status s)
{
    switch (s) {
    case LBF_OK: return "ok";
    case LBF_EINVAL: return "invalid argument";
    case LBF_ENOMEM: return "workspace too small";
    case LBF_EHIP: return "HIP runtime error";
    case LBF_ENOTCONV: return "not converged within the step budget";
    case LBF_EDIVERGED: return "diverged (non-finite values)";
    case LBF_ESTATE: return "call out of order";
    }
    return "unknown status";
}

const char *lbf_last_error(lbf_ctx ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

lbf_status lbf_params_default(lbf_params *p, int nx, int ny)
{
    if (!p) return LBF_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->nx = nx;
    p->ny = ny;
    p->real_bytes = 4;
    p->nspecies = 3;
    p->reaction_mode = 0;
    p->tau_f = 0.8;
    p->u0 = 0.05;
    p->tau_g = 0.8;
    p->c_in = 1.0;
    p->vel_scale = 1.0;
    p->flux_col = -1;
    return LBF_OK;
}

lbf_status lbf_create(const lbf_params *p, lbf_ctx *out)
{
    if (!out) return LBF_EINVAL;
    *out = nullptr;
    std::string why;
    lbf_status st = validate_params(p, why);
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return LBF_ENOMEM;
    c->err = why;
    *out = c;
    if (st != LBF_OK) return st;  // context still returned so lbf_last_error works
    c->p = *p;
    c->xf = p->flux_col == -1 ? p->nx - 3 : p->flux_col;
    c->cref = storage_shift(*p);
    c->L = make_launch(p->nx, p->ny, 256, 1);
    c->L.xcd_remap = !(p->flags & 1);
    layout(c);
    const bool ext = p->reaction_mode != 0 || p->boundary != 0;
    const bool vec = !ext && (p->variant == 2 || (p->variant == 0 && p->real_bytes == 8));
    if (vec) {
        const int V = 16 / p->real_bytes;
        c->Lv = make_launch(c->nxp / V, p->ny, p->tile_x > 0 ? p->tile_x : 64,
                            p->tile_y > 0 ? p->tile_y : 4);
        c->Lv.vec = true;
    } else {
        c->Lv = make_launch(p->nx, p->ny, p->tile_x > 0 ? p->tile_x : 256,
                            p->tile_y > 0 ? p->tile_y : 1);
    }
    c->Lv.xcd_remap = !(p->flags & 1);
    // Streaming (non-temporal) accesses pay off once the two ADR lattices no
    // longer fit the last-level cache; below that, cached accesses let steps
    // hit in it.
    const size_t adr_state = 2 * (size_t)p->nspecies * 5 * p->real_bytes * c->plane;
    bool nt = adr_state > NT_MIN_BYTES;
    if (p->flags & 64) nt = true;
    if (p->flags & 2) nt = false;
    c->Lv.nontemporal = c->L.nontemporal = nt;
    c->Lv.fp32_math = c->L.fp32_math = (p->flags & 16) != 0;
    c->Lv.mode = c->L.mode = p->reaction_mode;
    c->Lv.periodic = c->L.periodic = p->boundary == 1;
    c->Lv.wide = c->L.wide = wide_lattice(c->plane, p->real_bytes, p->flags);
    // untraced steps of the link-reaction channel run two per launch unless
    // flags bit 8 asks for one step per launch
    c->pair = !ext && !(p->flags & 256);
    if (c->pair) {
        int tx, ty;
        pair_tile(p->real_bytes, tx, ty);
        c->Lp = c->L;
        const Launch t = make_launch(p->nx, p->ny, tx, ty);
        c->Lp.tx = t.tx;
        c->Lp.ty = t.ty;
        c->Lp.gx = t.gx;
        c->Lp.gy = t.gy;
        c->Lp.vec = false;
        // flags bit 9: marching wavefronts instead of the LDS tile (FP32
        // storage with FP64 arithmetic and 32-bit offsets only)
        c->march = (p->flags & 512) && p->real_bytes == 4 && !c->Lp.fp32_math && !c->Lp.wide;
        if (c->march) c->Lm = march_launch(c->Lp, p->nx, p->ny, 22);
    }
    c->flow_fp32_math = (p->flags & (16 | 32)) != 0;
    // flow steps run two per launch (FP64 arithmetic, a channel of at least
    // FLOW_PAIR_MIN_NODES nodes) unless flags bit 8 asks for one per launch
    c->flow_pair = !(p->flags & 256) && p->boundary == 0 && !c->flow_fp32_math &&
                   (long)p->nx * p->ny >= FLOW_PAIR_MIN_NODES;
    if (c->flow_pair) {
        int tx, ty;
        pair_tile(p->real_bytes, tx, ty);
        c->Lfp = c->L;
        const Launch t = make_launch(p->nx, p->ny, tx, ty);
        c->Lfp.tx = t.tx;
        c->Lfp.ty = t.ty;
        c->Lfp.gx = t.gx;
        c->Lfp.gy = t.gy;
        c->Lfp.vec = false;
    }
    c->valid = true;
    return LBF_OK;
}

lbf_status lbf_workspace_bytes(lbf_ctx c, size_t *bytes)
{
    if (!c || !bytes) return LBF_EINVAL;
    if (!c->valid) return fail(c, LBF_EINVAL, "context was created with invalid parameters");
    *bytes = c->ws_need;
    return LBF_OK;
}

lbf_status lbf_bind(lbf_ctx c, void *ws, size_t bytes, void *stream)
{
    if (!c) return LBF_EINVAL;
    if (!c->valid) return fail(c, LBF_EINVAL, "context was created with invalid parameters");
    if (!ws) return fail(c, LBF_EINVAL, "workspace is NULL");
    if ((uintptr_t)ws % 256) return fail(c, LBF_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < c->ws_need) return fail(c, LBF_ENOMEM, "workspace smaller than lbf_workspace_bytes");
    clear_graphs(c);
    if (!c->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreate");
    }
    c->ws = (char *)ws;
    c->ws_bytes = bytes;
    c->stream = (hipStream_t)stream;
    c->geometry_set = c->rates_set = c->velocity_set = false;
    c->flow_steps = c->adr_steps = 0;
    c->adr_ready = false;
    return LBF_OK;
}

lbf_status lbf_set_geometry(lbf_ctx c, const uint8_t *type_dev)
{
    lbf_status st = check_ready(c, false);
    if (st != LBF_OK) return st;
    if (!type_dev) return fail(c, LBF_EINVAL, "node_type is NULL");
    const int nx = c->p.nx, ny = c->p.ny;
    // host-side check of the wall rows and the type values
    std::vector<uint8_t> t((size_t)nx * ny);
    hipError_t e = hipMemcpyAsync(t.data(), type_dev, t.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy node_type");
    if (c->p.boundary == 0)
        for (int x = 0; x < nx; ++x)
            if (t[x] == 0 || t[(size_t)(ny - 1) * nx + x] == 0)
                return fail(c, LBF_EINVAL, "rows 0 and ny-1 must be solid");
    for (uint8_t v : t)
        if (v > 3) return fail(c, LBF_EINVAL, "node_type values must be 0..3");
    e = launch_masks(type_dev, (uint8_t *)c->ptr(c->off.type), (uint8_t *)c->ptr(c->off.mask5),
                     (uint16_t *)c->ptr(c->off.mask9), nx, ny, c->nxp, c->p.nspecies,
                     c->p.boundary == 1, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "mask kernel");
    int *counter = (int *)c->ptr(c->off.counter);
    e = hipMemsetAsync(counter, 0, sizeof(int), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemsetAsync(counter)");
    e = launch_trace_list((const uint8_t *)c->ptr(c->off.mask5), (int32_t *)c->ptr(c->off.trace_idx),
                          (int32_t *)c->ptr(c->off.trace_nodes), counter, nx, ny, c->nxp, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "trace list kernel");
    int n = 0;
    e = hipMemcpyAsync(&n, counter, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read trace count");
    c->ntrace = n;
    c->geometry_set = true;
    c->rates_set = false;
    c->adr_ready = false;
    clear_graphs(c);
    return LBF_OK;
}

lbf_status lbf_set_rates(lbf_ctx c, const double *k_dev)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!k_dev) return fail(c, LBF_EINVAL, "k is NULL");
    const int nx = c->p.nx, ny = c->p.ny;
    std::vector<double> k((size_t)nx * ny);
    std::vector<uint8_t> t((size_t)c->plane);
    hipError_t e = hipMemcpyAsync(k.data(), k_dev, k.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t.data(), c->ptr(c->off.type), t.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy k");
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const uint8_t ty = t[(size_t)y * c->nxp + x];
            const double v = k[(size_t)y * nx + x];
            if ((ty == 2 || ty == 3) && !(v >= 0.0 && v <= 1.0))
                return fail(c, LBF_EINVAL, "rates at catalytic nodes must lie in [0, 1]");
        }
    e = launch_copy_rates(k_dev, (const uint8_t *)c->ptr(c->off.type), c->ptr(c->off.kr),
                          c->p.real_bytes, nx, ny, c->nxp, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "rate copy kernel");
    c->rates_set = true;
    return LBF_OK;
}

lbf_status lbf_flow_init(lbf_ctx c)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (c->p.boundary != 0) return fail(c, LBF_EINVAL, "the flow solve needs a channel (boundary 0)");
    c->fpar = 0;
    hipError_t e = launch_flow_init(c->p.real_bytes, flow_args<float>(c, 1), flow_args<double>(c, 1),
                                    c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "flow init kernel");
    c->flow_steps = 0;
    c->flow_ready = true;
    c->velocity_set = true;
    return LBF_OK;
}

lbf_status lbf_flow_run(lbf_ctx c, long nsteps)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->flow_ready) return fail(c, LBF_ESTATE, "call lbf_flow_init first");
    if (nsteps < 0) return fail(c, LBF_EINVAL, "nsteps < 0");
    long done = 0;
    while (done < nsteps) {
        const long n = std::min<long>(c->block_steps, nsteps - done);
        st = run_steps(c, KIND_FLOW, n);
        if (st != LBF_OK) return st;
        done += n;
        c->flow_steps += n;
    }
    c->adr_ready = false;
    return LBF_OK;
}

lbf_status lbf_flow_steady(lbf_ctx c, long max_steps, int check_every, double tol, long *steps_done,
                           double *residual)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->flow_ready) return fail(c, LBF_ESTATE, "call lbf_flow_init first");
    if (check_every < 1 || max_steps < 0) return fail(c, LBF_EINVAL, "bad step counts");
    const size_t ubytes = 2 * c->plane * c->p.real_bytes;
    hipError_t e = hipMemcpyAsync(c->ptr(c->off.uprev), c->ptr(c->off.u), ubytes,
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy u");
    long steps = 0;
    double res = INFINITY;
    bool conv = false;
    while (steps < max_steps) {
        const long n = std::min<long>(check_every, max_steps - steps);
        st = run_steps(c, KIND_FLOW, n);
        if (st != LBF_OK) return st;
        steps += n;
        c->flow_steps += n;
        if (tol > 0) {
            e = launch_du_max(c->p.real_bytes, c->ptr(c->off.u), c->ptr(c->off.uprev),
                              (const uint16_t *)c->ptr(c->off.mask9), c->plane,
                              (double *)c->ptr(c->off.partial), 1024,
                              (double *)c->ptr(c->off.obs) + 8, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "du reduction");
            double h[9];
            st = read_obs(c, h, 9);
            if (st != LBF_OK) return st;
            res = h[8];
            if (!std::isfinite(res)) return fail(c, LBF_EDIVERGED, "non-finite flow velocity");
            if (n == check_every && res <= tol * std::fabs(c->p.u0)) {
                conv = true;
                break;
            }
        }
    }
    if (tol <= 0) {
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    }
    if (steps_done) *steps_done = steps;
    if (residual) *residual = res;
    c->adr_ready = false;
    if (tol > 0 && !conv) return fail(c, LBF_ENOTCONV, "flow not converged within max_steps");
    return LBF_OK;
}

lbf_status lbf_get_velocity(lbf_ctx c, void *ux, void *uy)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->velocity_set) return fail(c, LBF_ESTATE, "no flow velocity yet");
    if (!ux || !uy) return fail(c, LBF_EINVAL, "NULL output");
    const size_t R = c->p.real_bytes;
    hipError_t e = launch_unpad(c->p.real_bytes, c->ptr(c->off.u), ux, c->p.nx, c->p.ny, c->nxp, c->stream);
    if (e == hipSuccess)
        e = launch_unpad(c->p.real_bytes, (char *)c->ptr(c->off.u) + c->plane * R, uy, c->p.nx,
                         c->p.ny, c->nxp, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "unpad velocity");
    return LBF_OK;
}

lbf_status lbf_set_velocity(lbf_ctx c, const void *ux, const void *uy)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!ux || !uy) return fail(c, LBF_EINVAL, "NULL input");
    const size_t R = c->p.real_bytes;
    hipError_t e = launch_pad(c->p.real_bytes, ux, c->ptr(c->off.u), c->p.nx, c->p.ny, c->nxp, c->stream);
    if (e == hipSuccess)
        e = launch_pad(c->p.real_bytes, uy, (char *)c->ptr(c->off.u) + c->plane * R, c->p.nx,
                       c->p.ny, c->nxp, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "pad velocity");
    c->velocity_set = true;
    c->adr_ready = false;
    return LBF_OK;
}

lbf_status lbf_adr_init(lbf_ctx c)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->rates_set) return fail(c, LBF_ESTATE, "rates not set");
    if (!c->velocity_set) return fail(c, LBF_ESTATE, "no flow velocity (run or import the flow)");
    hipError_t e = launch_velocity_handoff(c->p.real_bytes, c->ptr(c->off.u), c->ptr(c->off.ua),
                                           (const uint8_t *)c->ptr(c->off.mask5), c->p.vel_scale,
                                           c->plane, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "velocity handoff");
    c->gpar = 0;
    // the init kernel writes lattice 0 (its "src" argument is lattice 1)
    AdrArgs<float> af = adr_args<float>(c, 1);
    AdrArgs<double> ad = adr_args<double>(c, 1);
    e = launch_adr_init(c->p.real_bytes, c->p.nspecies, af, ad, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "ADR init kernel");
    c->adr_steps = 0;
    c->adr_ready = true;
    return LBF_OK;
}

lbf_status lbf_adr_run(lbf_ctx c, long max_steps, int check_every, double tol, long *steps_done)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->adr_ready) return fail(c, LBF_ESTATE, "call lbf_adr_init first");
    if (check_every < 1 || max_steps < 0) return fail(c, LBF_EINVAL, "bad step counts");
    if (tol > 0 && c->p.boundary != 0)
        return fail(c, LBF_EINVAL, "a periodic box has no outlet flux: use tol <= 0");
    long steps = 0;
    double prev = NAN;
    bool conv = false;
    while (steps < max_steps) {
        const long n = std::min<long>(check_every, max_steps - steps);
        // long blocks are replayed as graphs of at most block_steps steps
        long left = n;
        while (left > 0) {
            const long m = std::min<long>(left, c->block_steps);
            st = run_steps(c, KIND_ADR, m);
            if (st != LBF_OK) return st;
            left -= m;
            c->adr_steps += m;
        }
        steps += n;
        if (tol > 0) {
            double o[4];
            st = compute_fluxes(c, o);
            if (st != LBF_OK) return st;
            const double eps = efficiency_of(o, c->p.nspecies);
            if (steady_check(o, c->p.nspecies, o[3], eps, prev, tol)) {
                conv = true;
                break;
            }
            prev = eps;
        }
    }
    if (steps_done) *steps_done = steps;
    if (tol > 0 && !conv) return fail(c, LBF_ENOTCONV, "ADR not converged within max_steps");
    return LBF_OK;
}

lbf_status lbf_efficiency(lbf_ctx c, double *eps, double *N, double *inflow)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (c->p.boundary != 0) return fail(c, LBF_EINVAL, "a periodic box has no outlet flux");
    double o[4];
    st = compute_fluxes(c, o);
    if (st != LBF_OK) return st;
    if (N)
        for (int s = 0; s < c->p.nspecies; ++s) N[s] = o[s];
    if (inflow) *inflow = o[3];
    if (eps) *eps = efficiency_of(o, c->p.nspecies);
    return LBF_OK;
}

lbf_status lbf_get_concentration(lbf_ctx c, int species, void *out)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (species < 0 || species >= c->p.nspecies) return fail(c, LBF_EINVAL, "bad species index");
    if (!out) return fail(c, LBF_EINVAL, "NULL output");
    if (c->adr_steps < 1) return fail(c, LBF_ESTATE, "no ADR step taken yet");
    const int prev = c->gpar ^ 1;
    hipError_t e = launch_concentration(c->p.real_bytes, c->p.nspecies, species,
                                        adr_args<float>(c, prev), adr_args<double>(c, prev), out,
                                        c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "concentration kernel");
    return LBF_OK;
}

lbf_status lbf_adr_totals(lbf_ctx c, double *totals)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!totals) return fail(c, LBF_EINVAL, "NULL output");
    if (c->adr_steps < 1) return fail(c, LBF_ESTATE, "no ADR step taken yet");
    const int prev = c->gpar ^ 1;
    constexpr int NB = 256;  // blocks; 3 x NB partials fit the workspace partial block
    double *partial = (double *)c->ptr(c->off.partial);
    double *obs = (double *)c->ptr(c->off.obs);
    hipError_t e = launch_totals(c->p.real_bytes, c->p.nspecies, adr_args<float>(c, prev),
                                 adr_args<double>(c, prev), partial, NB, obs, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "totals kernel");
    return read_obs(c, totals, c->p.nspecies);
}

lbf_status lbf_adr_production(lbf_ctx c, double *rates)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!rates) return fail(c, LBF_EINVAL, "NULL output");
    if (c->adr_steps < 1) return fail(c, LBF_ESTATE, "no ADR step taken yet");
    const int prev = c->gpar ^ 1;
    constexpr int NB = 256;  // blocks; 2 x NB partials fit the workspace partial block
    double *partial = (double *)c->ptr(c->off.partial);
    double *obs = (double *)c->ptr(c->off.obs);
    hipError_t e = launch_production(c->p.real_bytes, c->p.nspecies, adr_args<float>(c, prev),
                                     adr_args<double>(c, prev), partial, NB, obs, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "production kernel");
    return read_obs(c, rates, c->p.nspecies - 1);
}

lbf_status lbf_adr_steps(lbf_ctx c, long *steps)
{
    if (!c || !steps) return LBF_EINVAL;
    *steps = c->adr_steps;
    return LBF_OK;
}

lbf_status lbf_state_bytes(lbf_ctx c, size_t *bytes)
{
    if (!c || !bytes) return LBF_EINVAL;
    if (!c->valid) return fail(c, LBF_EINVAL, "invalid context");
    *bytes = 2 * (size_t)c->p.nspecies * 5 * c->plane * c->p.real_bytes + 256;
    return LBF_OK;
}

lbf_status lbf_get_state(lbf_ctx c, void *dst)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!dst) return fail(c, LBF_EINVAL, "NULL output");
    if (!c->adr_ready) return fail(c, LBF_ESTATE, "no ADR state");
    const size_t L = (size_t)c->p.nspecies * 5 * c->plane * c->p.real_bytes;
    const int64_t hdr[4] = {c->adr_steps, (int64_t)c->p.nspecies, (int64_t)c->p.real_bytes,
                            (int64_t)c->plane};
    hipError_t e = hipMemcpyAsync(dst, c->ptr(c->off.g[c->gpar]), L, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char *)dst + L, c->ptr(c->off.g[c->gpar ^ 1]), L, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char *)dst + 2 * L, hdr, sizeof hdr, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "get_state copy");
    return LBF_OK;
}

lbf_status lbf_set_state(lbf_ctx c, const void *src)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!src) return fail(c, LBF_EINVAL, "NULL input");
    if (!c->velocity_set || !c->rates_set) return fail(c, LBF_ESTATE, "velocity and rates must be set");
    const size_t L = (size_t)c->p.nspecies * 5 * c->plane * c->p.real_bytes;
    int64_t hdr[4];
    hipError_t e = hipMemcpyAsync(hdr, (const char *)src + 2 * L, sizeof hdr, hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_state header");
    if (hdr[1] != c->p.nspecies || hdr[2] != c->p.real_bytes || hdr[3] != (int64_t)c->plane)
        return fail(c, LBF_EINVAL, "state blob does not match this context");
    if (c->adr_ready == false) {
        // the ADR velocity must be prepared as lbf_adr_init would
        e = launch_velocity_handoff(c->p.real_bytes, c->ptr(c->off.u), c->ptr(c->off.ua),
                                    (const uint8_t *)c->ptr(c->off.mask5), c->p.vel_scale, c->plane,
                                    c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "velocity handoff");
    }
    c->gpar = 0;
    e = hipMemcpyAsync(c->ptr(c->off.g[0]), src, L, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ptr(c->off.g[1]), (const char *)src + L, L, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_state copy");
    c->adr_steps = hdr[0];
    c->adr_ready = true;
    return LBF_OK;
}

static lbf_status time_steps(lbf_ctx c, int kind, long nsteps, double *ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    lbf_status st = LBF_OK;
    e = hipEventRecord(a, c->stream);
    long done = 0;
    while (e == hipSuccess && st == LBF_OK && done < nsteps) {
        const long n = std::min<long>(c->block_steps, nsteps - done);
        st = run_steps(c, kind, n);
        done += n;
        if (kind == KIND_ADR) c->adr_steps += n; else c->flow_steps += n;
    }
    if (e == hipSuccess) e = hipEventRecord(b, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != LBF_OK) return st;
    if (e != hipSuccess) return hip_fail(c, e, "timing events");
    if (ms) *ms = t;
    return LBF_OK;
}

lbf_status lbf_prepare_adr_steps(lbf_ctx c, long nsteps)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (nsteps < 1) return fail(c, LBF_EINVAL, "nsteps < 1");
    // lbf_adr_run and lbf_time_adr_steps split runs into blocks of at most
    // block_steps steps; blocks below GRAPH_MIN_STEPS launch directly
    const long n = std::min<long>(nsteps, c->block_steps);
    if (n < GRAPH_MIN_STEPS) return LBF_OK;
    for (int par = 0; par < 2; ++par) {
        hipGraphExec_t ex = nullptr;
        st = graph_of(c, KIND_ADR, n, par, &ex);
        if (st != LBF_OK) return st;
    }
    return LBF_OK;
}

lbf_status lbf_time_adr_steps(lbf_ctx c, long nsteps, double *ms)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->adr_ready) return fail(c, LBF_ESTATE, "call lbf_adr_init first");
    return time_steps(c, KIND_ADR, nsteps, ms);
}

lbf_status lbf_time_flow_steps(lbf_ctx c, long nsteps, double *ms)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->flow_ready) return fail(c, LBF_ESTATE, "call lbf_flow_init first");
    st = time_steps(c, KIND_FLOW, nsteps, ms);
    c->adr_ready = false;
    return st;
}

void lbf_destroy(lbf_ctx c)
{
    if (!c) return;
    clear_graphs(c);
    lbf::adjoint_release(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

lbf_status lbf_probe_copy(const void *src, void *dst, size_t nbytes, void *stream, double *ms)
{
    if (!src || !dst) return LBF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return LBF_EHIP;
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = launch_copy(src, dst, nbytes, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return LBF_EHIP;
    if (ms) *ms = t;
    return LBF_OK;
}

}  // extern "C"
