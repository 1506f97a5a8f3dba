// Host side of the 3D C ABI (include/lbf3d.h): validation, workspace layout,
// graph-captured step blocks, reductions read back to the host.
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "lbf3d_internal.hpp"

using lbf::Launch;
using namespace lbf::d3;

struct lbf3_ctx_s {
    lbf3_params p{};
    bool valid = false;
    std::string err;
    Geo g{};
    int xf = 0;
    double cref = 0;
    Launch L;
    bool flow_fp32_math = false;
    struct Offsets {
        size_t type, mask7, mask19, kr, f[2], u, uprev, ua, g[2], obs, partial;
    } off{};
    size_t ws_need = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr, cap_stream = nullptr;
    bool geometry_set = false, rates_set = false, velocity_set = false;
    bool flow_ready = false, adr_ready = false;
    int fpar = 0, gpar = 0;  // lattice holding the current post-collision state
    long flow_steps = 0, adr_steps = 0;
    long block_steps = 1000;
    std::map<std::tuple<int, long, int>, hipGraphExec_t> graphs;
    std::vector<uint8_t> type_host;  // node types, for the host-side rate check
    void *ptr(size_t o) const { return ws + o; }
};

namespace {

using Ctx = lbf3_ctx_s;
enum { KIND_ADR = 0, KIND_FLOW = 1 };
constexpr long GRAPH_MIN_STEPS = 8;
constexpr size_t NT_MIN_BYTES = (size_t)192 << 20;
constexpr int NB_PARTIAL = 256;

lbf_status fail(Ctx *c, lbf_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

lbf_status hip_fail(Ctx *c, hipError_t e, const char *what)
{
    return fail(c, LBF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

lbf_status validate(const lbf3_params *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return LBF_EINVAL; }
    if (p->nx < 8 || p->ny < 2 || p->nz < 2) { why = "need nx >= 8, ny >= 2, nz >= 2"; return LBF_EINVAL; }
    if ((double)p->nx * p->ny * p->nz > 2.0e9) { why = "lattice too large"; return LBF_EINVAL; }
    if (p->real_bytes != 4 && p->real_bytes != 8) { why = "real_bytes must be 4 or 8"; return LBF_EINVAL; }
    if (p->nspecies != 2 && p->nspecies != 3) { why = "nspecies must be 2 or 3"; return LBF_EINVAL; }
    if (!(p->tau_f > 0.5) || !std::isfinite(p->tau_f)) { why = "tau_f must be > 0.5"; return LBF_EINVAL; }
    if (!(p->tau_g > 0.5) || !std::isfinite(p->tau_g)) { why = "tau_g must be > 0.5"; return LBF_EINVAL; }
    if (!(std::fabs(p->force_x) <= 1e-3)) { why = "|force_x| must be <= 1e-3"; return LBF_EINVAL; }
    if (!std::isfinite(p->c_in)) { why = "c_in must be finite"; return LBF_EINVAL; }
    if (!(p->vel_scale >= 0) || !std::isfinite(p->vel_scale)) { why = "vel_scale must be >= 0"; return LBF_EINVAL; }
    if (p->flux_col != -1 && (p->flux_col < 1 || p->flux_col > p->nx - 2)) {
        why = "flux_col must be -1 or in [1, nx-2]";
        return LBF_EINVAL;
    }
    const int tx = p->tile_x > 0 ? p->tile_x : 64, ty = p->tile_y > 0 ? p->tile_y : 4;
    if (p->tile_x < 0 || p->tile_y < 0 || tx * ty > 1024 || (tx * ty) % 64 != 0) {
        why = "tile_x * tile_y must be a multiple of 64 and <= 1024";
        return LBF_EINVAL;
    }
    return LBF_OK;
}

void layout(Ctx *c)
{
    const lbf3_params &p = c->p;
    c->g.nx = p.nx;
    c->g.ny = p.ny;
    c->g.nz = p.nz;
    c->g.nxp = (int)lbf::align_up((size_t)p.nx, lbf::ROW_ALIGN);
    c->g.plane = (size_t)c->g.nxp * p.ny * p.nz;
    const size_t P = c->g.plane, R = (size_t)p.real_bytes;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = lbf::align_up(off + bytes, 256);
        return o;
    };
    c->off.type = take(P);
    c->off.mask7 = take(2 * P);
    c->off.mask19 = take(4 * P);
    c->off.kr = take(R * P);
    c->off.f[0] = take(19 * R * P);
    c->off.f[1] = take(19 * R * P);
    c->off.u = take(3 * R * P);
    c->off.uprev = take(3 * R * P);
    c->off.ua = take(3 * R * P);
    c->off.g[0] = take((size_t)p.nspecies * 7 * R * P);
    c->off.g[1] = take((size_t)p.nspecies * 7 * R * P);
    c->off.obs = take(16 * sizeof(double));
    c->off.partial = take(1024 * sizeof(double));
    c->ws_need = off;
}

template <typename Real>
AdrArgs3<Real> adr_args(Ctx *c, int src_buf)
{
    AdrArgs3<Real> a{};
    a.src = (const Real *)c->ptr(c->off.g[src_buf]);
    a.dst = (Real *)c->ptr(c->off.g[src_buf ^ 1]);
    a.ua = (const Real *)c->ptr(c->off.ua);
    a.mask7 = (const uint16_t *)c->ptr(c->off.mask7);
    a.type = (const uint8_t *)c->ptr(c->off.type);
    a.kr = (const Real *)c->ptr(c->off.kr);
    a.g = c->g;
    a.omega = 1.0 / c->p.tau_g;
    a.cin = c->p.c_in;
    a.cref = c->cref;
    a.L = c->L;
    return a;
}

template <typename Real>
FlowArgs3<Real> flow_args(Ctx *c, int src_buf)
{
    FlowArgs3<Real> a{};
    a.src = (const Real *)c->ptr(c->off.f[src_buf]);
    a.dst = (Real *)c->ptr(c->off.f[src_buf ^ 1]);
    a.mask19 = (const uint32_t *)c->ptr(c->off.mask19);
    a.u = (Real *)c->ptr(c->off.u);
    a.g = c->g;
    a.omega = 1.0 / c->p.tau_f;
    a.fx = c->p.force_x;
    a.L = c->L;
    a.L.fp32_math = c->flow_fp32_math;
    return a;
}

hipError_t enqueue_step(Ctx *c, int kind, int par, bool write_u, hipStream_t s)
{
    if (kind == KIND_ADR)
        return launch_adr_step3(c->p.real_bytes, c->p.nspecies, adr_args<float>(c, par),
                                adr_args<double>(c, par), s);
    return launch_flow_step3(c->p.real_bytes, write_u, flow_args<float>(c, par),
                             flow_args<double>(c, par), s);
}

// n consecutive steps; blocks of at least GRAPH_MIN_STEPS are captured once
// as a graph and replayed.  The velocity is written by the last flow step.
lbf_status run_steps(Ctx *c, int kind, long n)
{
    if (n <= 0) return LBF_OK;
    int &par = kind == KIND_ADR ? c->gpar : c->fpar;
    if (n < GRAPH_MIN_STEPS) {
        for (long i = 0; i < n; ++i) {
            hipError_t e = enqueue_step(c, kind, par, i == n - 1, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "step launch");
            par ^= 1;
        }
        return LBF_OK;
    }
    const auto key = std::make_tuple(kind, n, par);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
        int p = par;
        hipError_t le = hipSuccess;
        for (long i = 0; i < n && le == hipSuccess; ++i) {
            le = enqueue_step(c, kind, p, i == n - 1, c->cap_stream);
            p ^= 1;
        }
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(c->cap_stream, &gr);
        if (le != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return hip_fail(c, le, "step launch during capture");
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
        it = c->graphs.emplace(key, ex).first;
    }
    hipError_t e = hipGraphLaunch(it->second, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    if (n & 1) par ^= 1;
    return LBF_OK;
}

lbf_status run_blocks(Ctx *c, int kind, long n)
{
    while (n > 0) {
        const long m = std::min<long>(n, c->block_steps);
        lbf_status st = run_steps(c, kind, m);
        if (st != LBF_OK) return st;
        n -= m;
        (kind == KIND_ADR ? c->adr_steps : c->flow_steps) += m;
    }
    return LBF_OK;
}

void clear_graphs(Ctx *c)
{
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

lbf_status read_obs(Ctx *c, double *host, int n)
{
    hipError_t e = hipMemcpyAsync(host, c->ptr(c->off.obs), n * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "read back");
    return LBF_OK;
}

lbf_status check_ready(Ctx *c, bool need_geometry)
{
    if (!c) return LBF_EINVAL;
    if (!c->valid) return fail(c, LBF_EINVAL, "context was created with invalid parameters");
    if (!c->ws) return fail(c, LBF_ESTATE, "no workspace bound");
    if (need_geometry && !c->geometry_set) return fail(c, LBF_ESTATE, "geometry not set");
    return LBF_OK;
}

lbf_status fluxes(Ctx *c, double *out4)
{
    if (c->adr_steps < 1) return fail(c, LBF_ESTATE, "no ADR step taken yet");
    const int prev = c->gpar ^ 1;
    hipError_t e = launch_flux3(c->p.real_bytes, c->p.nspecies, adr_args<float>(c, prev),
                                adr_args<double>(c, prev), c->xf, (double *)c->ptr(c->off.obs),
                                c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "flux kernel");
    lbf_status st = read_obs(c, out4, 4);
    if (st != LBF_OK) return st;
    for (int s = 0; s < 4; ++s)
        if (!std::isfinite(out4[s])) return fail(c, LBF_EDIVERGED, "non-finite outlet flux");
    return LBF_OK;
}

double efficiency_of(const double *N, int ns)
{
    double den = 0.0;
    for (int s = 0; s < ns; ++s) den += N[s];
    return den != 0.0 ? N[ns - 1] / den : NAN;
}

lbf_status time_steps(Ctx *c, int kind, long n, double *ms)
{
    if (n < 1 || !ms) return fail(c, LBF_EINVAL, "need nsteps >= 1 and ms");
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(c, e, "hipEventCreate");
    }
    lbf_status st = LBF_OK;
    e = hipEventRecord(a, c->stream);
    if (e == hipSuccess) {
        st = run_blocks(c, kind, n);
        if (st == LBF_OK) e = hipEventRecord(b, c->stream);
        if (st == LBF_OK && e == hipSuccess) e = hipEventSynchronize(b);
        float f = 0;
        if (st == LBF_OK && e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
        *ms = f;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != LBF_OK) return st;
    if (e != hipSuccess) return hip_fail(c, e, "timing events");
    return LBF_OK;
}

}  // namespace

extern "C" {

lbf_status lbf3_params_default(lbf3_params *p, int nx, int ny, int nz)
{
    if (!p) return LBF_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->real_bytes = 4;
    p->nspecies = 3;
    p->tau_f = 0.8;
    p->force_x = 1e-6;
    p->tau_g = 0.8;
    p->c_in = 1.0;
    p->vel_scale = 1.0;
    p->flux_col = -1;
    return LBF_OK;
}

lbf_status lbf3_create(const lbf3_params *p, lbf3_ctx *out)
{
    if (!out) return LBF_EINVAL;
    *out = nullptr;
    std::string why;
    const lbf_status st = validate(p, why);
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return LBF_ENOMEM;
    c->err = why;
    *out = c;
    if (st != LBF_OK) return st;
    c->p = *p;
    c->xf = p->flux_col == -1 ? p->nx - 3 : p->flux_col;
    c->cref = p->real_bytes == 4 ? p->c_in : 0.0;
    layout(c);
    // 64 x 4 measured best on the 400 x 120 x 120 membrane (256 x 1: -7 %)
    c->L = lbf::make_launch(p->nx, p->ny * p->nz, p->tile_x > 0 ? p->tile_x : 64,
                            p->tile_y > 0 ? p->tile_y : 4);
    c->L.xcd_remap = !(p->flags & 1);
    const size_t adr_state = 2 * (size_t)p->nspecies * 7 * p->real_bytes * c->g.plane;
    bool nt = adr_state > NT_MIN_BYTES;
    if (p->flags & 64) nt = true;
    if (p->flags & 2) nt = false;
    c->L.nontemporal = nt;
    c->L.fp32_math = (p->flags & 16) != 0;
    c->flow_fp32_math = c->L.fp32_math;
    c->valid = true;
    return LBF_OK;
}

lbf_status lbf3_workspace_bytes(lbf3_ctx c, size_t *bytes)
{
    if (!c || !bytes) return LBF_EINVAL;
    if (!c->valid) return fail(c, LBF_EINVAL, "context was created with invalid parameters");
    *bytes = c->ws_need;
    return LBF_OK;
}

lbf_status lbf3_bind(lbf3_ctx c, void *ws, size_t bytes, void *stream)
{
    if (!c) return LBF_EINVAL;
    if (!c->valid) return fail(c, LBF_EINVAL, "context was created with invalid parameters");
    if (!ws) return fail(c, LBF_EINVAL, "workspace is NULL");
    if ((uintptr_t)ws % 256) return fail(c, LBF_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < c->ws_need) return fail(c, LBF_ENOMEM, "workspace smaller than lbf3_workspace_bytes");
    clear_graphs(c);
    if (!c->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreate");
    }
    c->ws = (char *)ws;
    c->ws_bytes = bytes;
    c->stream = (hipStream_t)stream;
    c->geometry_set = c->rates_set = c->velocity_set = false;
    c->flow_ready = c->adr_ready = false;
    c->flow_steps = c->adr_steps = 0;
    return LBF_OK;
}

lbf_status lbf3_set_geometry(lbf3_ctx c, const uint8_t *type_dev)
{
    lbf_status st = check_ready(c, false);
    if (st != LBF_OK) return st;
    if (!type_dev) return fail(c, LBF_EINVAL, "node_type is NULL");
    std::vector<uint8_t> t((size_t)c->p.nx * c->p.ny * c->p.nz);
    hipError_t e = hipMemcpyAsync(t.data(), type_dev, t.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy node_type");
    for (uint8_t v : t)
        if (v > 3) return fail(c, LBF_EINVAL, "node_type values must be 0..3");
    e = launch_masks3(type_dev, (uint8_t *)c->ptr(c->off.type), (uint16_t *)c->ptr(c->off.mask7),
                      (uint32_t *)c->ptr(c->off.mask19), c->g, c->p.nspecies, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "mask kernel");
    c->type_host.swap(t);
    c->geometry_set = true;
    c->rates_set = c->flow_ready = c->adr_ready = c->velocity_set = false;
    clear_graphs(c);
    return LBF_OK;
}

lbf_status lbf3_set_rates(lbf3_ctx c, const double *k_dev)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!k_dev) return fail(c, LBF_EINVAL, "k is NULL");
    const size_t n = (size_t)c->p.nx * c->p.ny * c->p.nz;
    std::vector<double> k(n);
    hipError_t e = hipMemcpyAsync(k.data(), k_dev, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy k");
    e = launch_copy_rates3(k_dev, (const uint8_t *)c->ptr(c->off.type), c->ptr(c->off.kr),
                           c->p.real_bytes, c->g, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "rate kernel");
    for (size_t i = 0; i < n; ++i)
        if (c->type_host[i] >= 2 && !(k[i] >= 0.0 && k[i] <= 1.0))
            return fail(c, LBF_EINVAL, "rates at catalytic nodes must lie in [0, 1]");
    c->rates_set = true;
    c->adr_ready = false;
    return LBF_OK;
}

lbf_status lbf3_flow_init(lbf3_ctx c)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    c->fpar = 0;
    hipError_t e = launch_flow_init3(c->p.real_bytes, flow_args<float>(c, 1), flow_args<double>(c, 1),
                                     c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "flow init kernel");
    c->flow_steps = 0;
    c->flow_ready = c->velocity_set = true;
    c->adr_ready = false;
    return LBF_OK;
}

lbf_status lbf3_flow_run(lbf3_ctx c, long nsteps)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->flow_ready) return fail(c, LBF_ESTATE, "call lbf3_flow_init first");
    if (nsteps < 0) return fail(c, LBF_EINVAL, "nsteps < 0");
    c->adr_ready = false;
    return run_blocks(c, KIND_FLOW, nsteps);
}

lbf_status lbf3_flow_steady(lbf3_ctx c, long max_steps, int check_every, double tol,
                            long *steps_done, double *residual)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->flow_ready) return fail(c, LBF_ESTATE, "call lbf3_flow_init first");
    if (check_every < 1 || max_steps < 0) return fail(c, LBF_EINVAL, "bad step counts");
    c->adr_ready = false;
    const size_t ubytes = 3 * c->g.plane * c->p.real_bytes;
    hipError_t e = hipMemcpyAsync(c->ptr(c->off.uprev), c->ptr(c->off.u), ubytes,
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy u");
    long steps = 0;
    double res = INFINITY;
    bool conv = false;
    while (steps < max_steps) {
        const long n = std::min<long>(check_every, max_steps - steps);
        st = run_blocks(c, KIND_FLOW, n);
        if (st != LBF_OK) return st;
        steps += n;
        if (tol > 0) {
            e = launch_du_max3(c->p.real_bytes, c->ptr(c->off.u), c->ptr(c->off.uprev),
                               (const uint32_t *)c->ptr(c->off.mask19), c->g.plane,
                               (double *)c->ptr(c->off.partial), NB_PARTIAL,
                               (double *)c->ptr(c->off.obs), c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "du reduction");
            double h[2];
            st = read_obs(c, h, 2);
            if (st != LBF_OK) return st;
            res = h[0];
            if (!std::isfinite(res)) return fail(c, LBF_EDIVERGED, "non-finite flow velocity");
            if (n == check_every && res <= tol * h[1]) {
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
    if (tol > 0 && !conv) return fail(c, LBF_ENOTCONV, "flow not converged within max_steps");
    return LBF_OK;
}

lbf_status lbf3_get_velocity(lbf3_ctx c, void *ux, void *uy, void *uz)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->velocity_set) return fail(c, LBF_ESTATE, "no flow velocity yet");
    if (!ux || !uy || !uz) return fail(c, LBF_EINVAL, "NULL output");
    // the three components go to one scratch block (the previous-velocity
    // buffer is free outside lbf3_flow_steady), then to the caller's arrays
    const size_t n = (size_t)c->p.nx * c->p.ny * c->p.nz, R = c->p.real_bytes;
    char *tmp = (char *)c->ptr(c->off.uprev);
    hipError_t e = launch_unpad3(c->p.real_bytes, c->ptr(c->off.u), tmp, c->g, c->stream);
    void *outs[3] = {ux, uy, uz};
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        e = hipMemcpyAsync(outs[k], tmp + k * n * R, n * R, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "velocity copy");
    return LBF_OK;
}

lbf_status lbf3_set_velocity(lbf3_ctx c, const void *ux, const void *uy, const void *uz)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!ux || !uy || !uz) return fail(c, LBF_EINVAL, "NULL input");
    const size_t n = (size_t)c->p.nx * c->p.ny * c->p.nz, R = c->p.real_bytes;
    char *tmp = (char *)c->ptr(c->off.uprev);
    const void *ins[3] = {ux, uy, uz};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        e = hipMemcpyAsync(tmp + k * n * R, ins[k], n * R, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_pad3(c->p.real_bytes, tmp, c->ptr(c->off.u), (const uint8_t *)c->ptr(c->off.type),
                        c->g, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "velocity import");
    c->velocity_set = true;
    c->flow_ready = false;
    c->adr_ready = false;
    return LBF_OK;
}

lbf_status lbf3_adr_init(lbf3_ctx c)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->rates_set) return fail(c, LBF_ESTATE, "rates not set");
    if (!c->velocity_set) return fail(c, LBF_ESTATE, "no flow velocity (run or import the flow)");
    hipError_t e = launch_velocity_handoff3(c->p.real_bytes, c->ptr(c->off.u), c->ptr(c->off.ua),
                                            (const uint16_t *)c->ptr(c->off.mask7), c->g.plane,
                                            c->p.vel_scale, c->stream);
    c->gpar = 0;
    if (e == hipSuccess)
        e = launch_adr_init3(c->p.real_bytes, c->p.nspecies, adr_args<float>(c, 1),
                             adr_args<double>(c, 1), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "ADR init kernels");
    c->adr_steps = 0;
    c->adr_ready = true;
    return LBF_OK;
}

lbf_status lbf3_adr_run(lbf3_ctx c, long max_steps, int check_every, double tol, long *steps_done)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->adr_ready) return fail(c, LBF_ESTATE, "call lbf3_adr_init first");
    if (check_every < 1 || max_steps < 0) return fail(c, LBF_EINVAL, "bad step counts");
    long steps = 0;
    double prev = NAN;
    bool conv = false;
    while (steps < max_steps) {
        const long n = std::min<long>(check_every, max_steps - steps);
        st = run_blocks(c, KIND_ADR, n);
        if (st != LBF_OK) return st;
        steps += n;
        if (tol > 0) {
            double o[4];
            st = fluxes(c, o);
            if (st != LBF_OK) return st;
            const double eps = efficiency_of(o, c->p.nspecies);
            if (lbf::steady_check(o, c->p.nspecies, o[3], eps, prev, tol)) {
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

lbf_status lbf3_efficiency(lbf3_ctx c, double *eps, double *N, double *inflow)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    double o[4];
    st = fluxes(c, o);
    if (st != LBF_OK) return st;
    if (N)
        for (int s = 0; s < c->p.nspecies; ++s) N[s] = o[s];
    if (inflow) *inflow = o[3];
    if (eps) *eps = efficiency_of(o, c->p.nspecies);
    return LBF_OK;
}

lbf_status lbf3_get_concentration(lbf3_ctx c, int species, void *out)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (species < 0 || species >= c->p.nspecies) return fail(c, LBF_EINVAL, "bad species index");
    if (!out) return fail(c, LBF_EINVAL, "NULL output");
    if (c->adr_steps < 1) return fail(c, LBF_ESTATE, "no ADR step taken yet");
    const int prev = c->gpar ^ 1;
    hipError_t e = launch_concentration3(c->p.real_bytes, c->p.nspecies, species,
                                         adr_args<float>(c, prev), adr_args<double>(c, prev), out,
                                         c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "concentration kernel");
    return LBF_OK;
}

lbf_status lbf3_adr_totals(lbf3_ctx c, double *totals)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!totals) return fail(c, LBF_EINVAL, "NULL output");
    if (c->adr_steps < 1) return fail(c, LBF_ESTATE, "no ADR step taken yet");
    const int prev = c->gpar ^ 1;
    hipError_t e = launch_totals3(c->p.real_bytes, c->p.nspecies, adr_args<float>(c, prev),
                                  adr_args<double>(c, prev), (double *)c->ptr(c->off.partial),
                                  NB_PARTIAL, (double *)c->ptr(c->off.obs), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "totals kernel");
    return read_obs(c, totals, c->p.nspecies);
}

lbf_status lbf3_time_adr_steps(lbf3_ctx c, long nsteps, double *ms)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->adr_ready) return fail(c, LBF_ESTATE, "call lbf3_adr_init first");
    return time_steps(c, KIND_ADR, nsteps, ms);
}

lbf_status lbf3_time_flow_steps(lbf3_ctx c, long nsteps, double *ms)
{
    lbf_status st = check_ready(c, true);
    if (st != LBF_OK) return st;
    if (!c->flow_ready) return fail(c, LBF_ESTATE, "call lbf3_flow_init first");
    c->adr_ready = false;
    return time_steps(c, KIND_FLOW, nsteps, ms);
}

const char *lbf3_last_error(lbf3_ctx c) { return c ? c->err.c_str() : "NULL context"; }

void lbf3_destroy(lbf3_ctx c)
{
    if (!c) return;
    clear_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

}  // extern "C"
