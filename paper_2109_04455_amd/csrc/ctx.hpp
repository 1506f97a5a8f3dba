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
    lbf::Launch L;

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

lbf_status fail(Ctx *c, lbf_status s, const std::string &msg);
lbf_status hip_fail(Ctx *c, hipError_t e, const char *what);
lbf_status check_ready(Ctx *c, bool need_geometry);
lbf_status run_steps(Ctx *c, int kind, long n);
lbf_status compute_fluxes(Ctx *c, double *out4);
double efficiency_of(const double *N, int ns);
hipError_t enqueue_adr_step(Ctx *c, int src_buf, hipStream_t s, void *trace_slot);
template <typename Real>
AdrArgs<Real> adr_args(Ctx *c, int src_buf);
void adjoint_release(Ctx *c);

}  // namespace lbf
