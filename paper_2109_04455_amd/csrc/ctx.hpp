// Context of one lattice (the opaque lbf_ctx of the C ABI).
#pragma once

#include <map>
#include <string>
#include <tuple>

#include "lbf_internal.hpp"

struct lbf_ctx_s {
    lbf_params p{};
    bool valid = false;
    std::string err;

    // geometry of the padded lattice
    int nxp = 0;
    size_t plane = 0;  // ny * nxp
    int xf = 0;        // outlet flux column
    double cref = 0;   // storage shift of species A
    lbf::Launch L;   // one node per thread
    lbf::Launch Lv;  // ADR step launch (vectorised or not, per params.variant)
    lbf::Launch Lp;  // two-step ADR launch (when `pair`)
    lbf::Launch Lm;  // marching two-step launch (when `march`)
    bool pair = false;  // untraced ADR steps run two per launch
    bool march = false;  // ... by the marching kernel instead of the LDS tile
    lbf::Launch Lfp;  // two-step flow launch (when `flow_pair`)
    bool flow_pair = false;  // flow steps run two per launch
    bool flow_fp32_math = false;  // flow step computes in FP32 (FP32 storage)

    // workspace (caller-owned) and its layout
    struct Offsets {
        size_t type, mask5, mask9, trace_idx, trace_nodes, kr;
        size_t f[2], u, uprev, ua, g[2], obs, partial, counter;
    } off{};
    size_t ws_need = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // used only to capture graphs

    void *ptr(size_t o) const { return ws + o; }

    // state
    bool geometry_set = false, rates_set = false, velocity_set = false;
    bool flow_ready = false, adr_ready = false;
    int fpar = 0;  // f[fpar] holds the current post-collision flow state
    int gpar = 0;  // g[gpar] holds the current post-collision ADR state
    long flow_steps = 0, adr_steps = 0;
    int ntrace = 0;  // fluid nodes next to catalytic nodes

    long block_steps = 1000;  // longest captured graph
    std::map<std::tuple<int, long, int>, hipGraphExec_t> graphs;

    // adjoint graph cache etc.
    void *adj = nullptr;
};

namespace lbf {

using Ctx = lbf_ctx_s;

enum { KIND_ADR = 0, KIND_FLOW = 1 };
constexpr long GRAPH_MIN_STEPS = 8;
// Above this size of the two ADR lattices the population accesses stream
// (non-temporal) by default: the 256 MiB last-level cache no longer holds a
// step's working set.
constexpr size_t NT_MIN_BYTES = (size_t)192 << 20;

// Population blocks (the 9 flow planes, a species' 5 ADR planes, the 2
// velocity planes) are addressed with 32-bit byte offsets while the largest,
// the flow lattice, stays below 4 GiB; beyond that, or with flags bit 7, the
// node updates use 64-bit offsets.
inline bool wide_lattice(size_t plane, int real_bytes, int flags)
{
    return (flags & 128) || 9 * plane * (size_t)real_bytes > (size_t)UINT32_MAX;
}

lbf_status fail(Ctx *c, lbf_status s, const std::string &msg);
lbf_status validate_params(const lbf_params *p, std::string &why);
void layout(Ctx *c);
lbf_status hip_fail(Ctx *c, hipError_t e, const char *what);
lbf_status check_ready(Ctx *c, bool need_geometry);
lbf_status run_steps(Ctx *c, int kind, long n);
lbf_status compute_fluxes(Ctx *c, double *out4);
double efficiency_of(const double *N, int ns);
hipError_t enqueue_adr_step(Ctx *c, int src_buf, hipStream_t s, void *trace_slot);
hipError_t enqueue_adr_pair(Ctx *c, int src_buf, hipStream_t s);
void adjoint_release(Ctx *c);

// Two flow steps per launch (kernels_flow.hip): a.L is the two-step tiling.
hipError_t launch_flow_pair(int real_bytes, bool write_u, const FlowArgs<float> &af,
                            const FlowArgs<double> &ad, hipStream_t s);
// Flow steps run two per launch on lattices of at least this many nodes
// (below it a launch covers a few blocks and one row per thread is kept).
constexpr long FLOW_PAIR_MIN_NODES = 1L << 18;

// Kernel argument blocks for the context's own lattices.
template <typename Real>
inline AdrArgs<Real> adr_args(Ctx *c, int src_buf)
{
    AdrArgs<Real> a{};
    a.src = (const Real *)c->ptr(c->off.g[src_buf]);
    a.dst = (Real *)c->ptr(c->off.g[src_buf ^ 1]);
    a.ua = (const Real *)c->ptr(c->off.ua);
    a.mask5 = (const uint8_t *)c->ptr(c->off.mask5);
    a.type = (const uint8_t *)c->ptr(c->off.type);
    a.kr = (const Real *)c->ptr(c->off.kr);
    a.trace_idx = (const int32_t *)c->ptr(c->off.trace_idx);
    a.trace = nullptr;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nxp = c->nxp;
    a.plane = c->plane;
    a.omega = 1.0 / c->p.tau_g;
    a.cin = c->p.c_in;
    a.cref = c->cref;
    a.L = c->L;
    return a;
}

template <typename Real>
inline FlowArgs<Real> flow_args(Ctx *c, int src_buf)
{
    FlowArgs<Real> a{};
    a.src = (const Real *)c->ptr(c->off.f[src_buf]);
    a.dst = (Real *)c->ptr(c->off.f[src_buf ^ 1]);
    a.mask9 = (const uint16_t *)c->ptr(c->off.mask9);
    a.u = (Real *)c->ptr(c->off.u);
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nxp = c->nxp;
    a.plane = c->plane;
    a.omega = 1.0 / c->p.tau_f;
    a.u0 = c->p.u0;
    a.L = c->L;
    a.L.fp32_math = c->flow_fp32_math;
    return a;
}



}  // namespace lbf
