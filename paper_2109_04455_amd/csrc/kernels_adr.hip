// D2Q5 advection-diffusion-reaction kernels: one fused pull-stream /
// collide / react step for all species of a node per thread.
//
// Storage: post-collision populations of S species as a structure of arrays
// [S][5][ny][nxp] (x contiguous, rows padded to 64 elements).  Species A is
// stored shifted, h_i = g_i - w_i cref (cref = c_in in FP32), so the small
// depletion of A keeps its relative precision; B and C are stored as is.
// The shift is exact algebra: bounce-back keeps h, the anti-bounce-back
// inlet becomes h_E = -h*_W + 2 w (c_in - cref), the zero-gradient outlet
// h_W = -h*_E + 2 w sum_j h*_j, and the collision
// h* = h - omega (h - w_i p_i cref - e_i delta), with delta = sum_i h_i,
// e_i = w_i (1 + p_i), p_i = 3 c.u + 4.5 (c.u)^2 - 1.5 u.u.
//
// Paper: Sec. "Lattice-Boltzmann for Advection-Diffusion-Reaction" (Eqs.
// LBE_ADE, BGK, second-order equilibrium with cs^2 = 1/3, source_lbm applied
// only to populations that stream into a reactive boundary node) and Sec.
// "Boundary conditions and flux computation in ADE" (Eq. BC, inlet C_A = 1
// with bounce-back for the other species, outlet C_w = C_b, outflux plane
// two nodes before the right boundary).
#include "stencil.hpp"

namespace lbf {
namespace {

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
template <typename Real>
__device__ __forceinline__ void pull5(const Real *__restrict__ src, size_t P, size_t id, int x,
                                      int nx, int nxp, unsigned m, bool species_a, Real inlet_e,
                                      Real (&h)[5])
{
    h[0] = src[id];
    // E arrives from x - 1
    if (x == 0)
        h[DE] = species_a ? inlet_e - src[DW * P + id] : src[DW * P + id];
    else if (m & BIT_W)
        h[DE] = src[DW * P + id];
    else
        h[DE] = src[DE * P + id - 1];
    // N arrives from y - 1
    h[DN] = (m & BIT_S) ? src[DS * P + id] : src[DN * P + id - nxp];
    // W arrives from x + 1
    if (x == nx - 1) {
        const Real sum = src[id] + src[DE * P + id] + src[DN * P + id] + src[DW * P + id] +
                         src[DS * P + id];
        h[DW] = Real(2) * w5<Real>(DW) * sum - src[DE * P + id];
    } else if (m & BIT_E) {
        h[DW] = src[DE * P + id];
    } else {
        h[DW] = src[DW * P + id + 1];
    }
    // S arrives from y + 1
    h[DS] = (m & BIT_N) ? src[DN * P + id] : src[DS * P + id + nxp];
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

// Collide + react + store for one node given its gathered populations.
template <typename Real, int S, bool TRACE>
__device__ __forceinline__ void collide_react_store(const AdrArgs<Real> &a, size_t id, unsigned m,
                                                    Real (&h)[S][5])
{
    const size_t P = a.plane;
    const Real u = a.ua[id], v = a.ua[P + id];
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
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 5; ++i) a.dst[(s * 5 + i) * P + id] = h[s][i];
}

template <typename Real, int S, bool TRACE>
__global__ __launch_bounds__(1024) void k_adr_step(AdrArgs<Real> a)
{
    int x, y;
    tile_coords(a.L, x, y);
    if (x >= a.nx || y >= a.ny) return;
    const size_t id = (size_t)y * a.nxp + x;
    const unsigned m = a.mask5[id];
    if (m == MASK5_SOLID) return;
    const size_t P = a.plane;
    const Real inlet_e = Real(2) * w5<Real>(DE) * (a.cin - a.cref);
    Real h[S][5];
#pragma unroll
    for (int s = 0; s < S; ++s)
        pull5(a.src + (size_t)s * 5 * P, P, id, x, a.nx, a.nxp, m, s == 0, inlet_e, h[s]);
    collide_react_store<Real, S, TRACE>(a, id, m, h);
}

// Initial state: A at equilibrium with C = c_in and the ADR velocity, B = C = 0,
// then one collision + reaction (the stored state is post-collision).
template <typename Real, int S>
__global__ __launch_bounds__(1024) void k_adr_init(AdrArgs<Real> a)
{
    int x, y;
    tile_coords(a.L, x, y);
    if (x >= a.nx || y >= a.ny) return;
    const size_t id = (size_t)y * a.nxp + x;
    const size_t P = a.plane;
    const unsigned m = a.mask5[id];
    if (m == MASK5_SOLID) {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < 5; ++i) a.dst[(s * 5 + i) * P + id] = 0;
        return;
    }
    Real p[5];
    eq_factors(a.ua[id], a.ua[P + id], p);
    Real h[S][5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        // g_A = w_i c_in (1 + p_i), stored as g_A - w_i cref
        h[0][i] = w5<Real>(i) * (a.cin * p[i] + (a.cin - a.cref));
#pragma unroll
        for (int s = 1; s < S; ++s) h[s][i] = 0;
    }
    collide_react_store<Real, S, false>(a, id, m, h);
}

// Concentration of one species after the last step: gather from the
// previous post-collision lattice exactly as the step does, then sum.
template <typename Real>
__global__ __launch_bounds__(1024) void k_concentration(AdrArgs<Real> a, int species, Real *out)
{
    int x, y;
    tile_coords(a.L, x, y);
    if (x >= a.nx || y >= a.ny) return;
    const size_t id = (size_t)y * a.nxp + x;
    const unsigned m = a.mask5[id];
    Real c = 0;
    if (m != MASK5_SOLID) {
        Real h[5];
        const Real inlet_e = Real(2) * w5<Real>(DE) * (a.cin - a.cref);
        pull5(a.src + (size_t)species * 5 * a.plane, a.plane, id, x, a.nx, a.nxp, m, species == 0,
              inlet_e, h);
        c = (species == 0 ? a.cref : Real(0)) + (h[0] + h[1] + h[2] + h[3] + h[4]);
    }
    out[(size_t)y * a.nx + x] = c;
}

// Concentrations (C_A, C_B) at the trace nodes after the last step.
template <typename Real, int S>
__global__ __launch_bounds__(256) void k_trace_conc(AdrArgs<Real> a, const int32_t *nodes, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const size_t id = nodes[t];
    const int x = (int)(id % a.nxp);
    const unsigned m = a.mask5[id];
    const Real inlet_e = Real(2) * w5<Real>(DE) * (a.cin - a.cref);
    Real h[5];
    pull5(a.src, a.plane, id, x, a.nx, a.nxp, m, true, inlet_e, h);
    a.trace[2 * t] = a.cref + (h[0] + h[1] + h[2] + h[3] + h[4]);
    Real cb = 0;
    if (S == 3) {
        pull5(a.src + 5 * a.plane, a.plane, id, x, a.nx, a.nxp, m, false, inlet_e, h);
        cb = h[0] + h[1] + h[2] + h[3] + h[4];
    }
    a.trace[2 * t + 1] = cb;
}

// Outlet fluxes and inlet flux of the last streaming, from the previous
// post-collision lattice: N_s = sum_y [g*_E(xf) - g*_W(xf+1)] over rows where
// both nodes are fluid; inflow_A = sum_y [2 w c_in - 2 g*_W,A(0)].
// One block, FP64 accumulation, fixed reduction order (deterministic).
template <typename Real>
__global__ __launch_bounds__(256) void k_flux(const Real *src, const uint8_t *mask5, int ns, int nx,
                                              int ny, int nxp, size_t P, int xf, double cin,
                                              double cref, double *out)
{
    __shared__ double sm[4][256];
    double acc[4] = {0, 0, 0, 0};
    for (int y = threadIdx.x; y < ny; y += blockDim.x) {
        const size_t a = (size_t)y * nxp + xf, b = a + 1;
        if (mask5[a] != MASK5_SOLID && mask5[b] != MASK5_SOLID)
            for (int s = 0; s < ns; ++s)
                acc[s] += (double)src[(s * 5 + DE) * P + a] - (double)src[(s * 5 + DW) * P + b];
        const size_t i0 = (size_t)y * nxp;
        if (mask5[i0] != MASK5_SOLID)
            acc[3] += 2.0 * (1.0 / 6.0) * (cin - cref) - 2.0 * (double)src[DW * P + i0];
    }
    for (int s = 0; s < 4; ++s) sm[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int s = 0; s < 4; ++s) sm[s][threadIdx.x] += sm[s][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int s = 0; s < 4; ++s) out[s] = sm[s][0];
}

template <typename Real>
__global__ void k_velocity_handoff(const Real *u, Real *ua, const uint8_t *mask5, double scale,
                                   size_t plane)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * plane;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t id = i < plane ? i : i - plane;
        ua[i] = mask5[id] == MASK5_SOLID ? Real(0) : Real(scale * (double)u[i]);
    }
}

template <typename Real>
__global__ void k_unpad(const Real *src, Real *dst, int nx, int ny, int nxp)
{
    const size_t n = (size_t)nx * ny;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[(i / nx) * nxp + i % nx];
}

template <typename Real>
__global__ void k_pad(const Real *src, Real *dst, int nx, int ny, int nxp)
{
    const size_t n = (size_t)nxp * ny;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t x = i % nxp, y = i / nxp;
        dst[i] = x < (size_t)nx ? src[y * nx + x] : Real(0);
    }
}

template <typename Real>
hipError_t step_dispatch(int ns, bool trace, const AdrArgs<Real> &a, hipStream_t s)
{
    const dim3 g = a.L.grid(), b = a.L.block();
    if (ns == 2) {
        if (trace)
            hipLaunchKernelGGL((k_adr_step<Real, 2, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_adr_step<Real, 2, false>), g, b, 0, s, a);
    } else {
        if (trace)
            hipLaunchKernelGGL((k_adr_step<Real, 3, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_adr_step<Real, 3, false>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adr_step(int real_bytes, int ns, bool trace, const AdrArgs<float> &af,
                           const AdrArgs<double> &ad, hipStream_t s)
{
    return real_bytes == 4 ? step_dispatch(ns, trace, af, s) : step_dispatch(ns, trace, ad, s);
}

hipError_t launch_adr_init(int real_bytes, int ns, const AdrArgs<float> &af,
                           const AdrArgs<double> &ad, hipStream_t s)
{
    if (real_bytes == 4) {
        if (ns == 2)
            hipLaunchKernelGGL((k_adr_init<float, 2>), af.L.grid(), af.L.block(), 0, s, af);
        else
            hipLaunchKernelGGL((k_adr_init<float, 3>), af.L.grid(), af.L.block(), 0, s, af);
    } else {
        if (ns == 2)
            hipLaunchKernelGGL((k_adr_init<double, 2>), ad.L.grid(), ad.L.block(), 0, s, ad);
        else
            hipLaunchKernelGGL((k_adr_init<double, 3>), ad.L.grid(), ad.L.block(), 0, s, ad);
    }
    return hipGetLastError();
}

hipError_t launch_flux(int real_bytes, int ns, const void *src, const uint8_t *mask5, int nx, int ny,
                       int nxp, size_t plane, int xf, double cin, double cref, double *out,
                       hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_flux<float>, dim3(1), dim3(256), 0, s, (const float *)src, mask5, ns,
                           nx, ny, nxp, plane, xf, cin, cref, out);
    else
        hipLaunchKernelGGL(k_flux<double>, dim3(1), dim3(256), 0, s, (const double *)src, mask5, ns,
                           nx, ny, nxp, plane, xf, cin, cref, out);
    return hipGetLastError();
}

hipError_t launch_concentration(int real_bytes, int ns, int species, const AdrArgs<float> &af,
                                const AdrArgs<double> &ad, void *out, hipStream_t s)
{
    (void)ns;
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_concentration<float>, af.L.grid(), af.L.block(), 0, s, af, species,
                           (float *)out);
    else
        hipLaunchKernelGGL(k_concentration<double>, ad.L.grid(), ad.L.block(), 0, s, ad, species,
                           (double *)out);
    return hipGetLastError();
}

hipError_t launch_trace_conc(int real_bytes, int ns, const AdrArgs<float> &af,
                             const AdrArgs<double> &ad, const int32_t *trace_nodes, int ntrace,
                             hipStream_t s)
{
    if (ntrace <= 0) return hipSuccess;
    const dim3 g((ntrace + 255) / 256), b(256);
    if (real_bytes == 4) {
        if (ns == 2)
            hipLaunchKernelGGL((k_trace_conc<float, 2>), g, b, 0, s, af, trace_nodes, ntrace);
        else
            hipLaunchKernelGGL((k_trace_conc<float, 3>), g, b, 0, s, af, trace_nodes, ntrace);
    } else {
        if (ns == 2)
            hipLaunchKernelGGL((k_trace_conc<double, 2>), g, b, 0, s, ad, trace_nodes, ntrace);
        else
            hipLaunchKernelGGL((k_trace_conc<double, 3>), g, b, 0, s, ad, trace_nodes, ntrace);
    }
    return hipGetLastError();
}

hipError_t launch_velocity_handoff(int real_bytes, const void *u, void *ua, const uint8_t *mask5,
                                   double vel_scale, size_t plane, hipStream_t s)
{
    const dim3 g(1024), b(256);
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_velocity_handoff<float>, g, b, 0, s, (const float *)u, (float *)ua,
                           mask5, vel_scale, plane);
    else
        hipLaunchKernelGGL(k_velocity_handoff<double>, g, b, 0, s, (const double *)u, (double *)ua,
                           mask5, vel_scale, plane);
    return hipGetLastError();
}

hipError_t launch_unpad(int real_bytes, const void *src, void *dst, int nx, int ny, int nxp,
                        hipStream_t s)
{
    const dim3 g(1024), b(256);
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_unpad<float>, g, b, 0, s, (const float *)src, (float *)dst, nx, ny, nxp);
    else
        hipLaunchKernelGGL(k_unpad<double>, g, b, 0, s, (const double *)src, (double *)dst, nx, ny,
                           nxp);
    return hipGetLastError();
}

hipError_t launch_pad(int real_bytes, const void *src, void *dst, int nx, int ny, int nxp,
                      hipStream_t s)
{
    const dim3 g(1024), b(256);
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_pad<float>, g, b, 0, s, (const float *)src, (float *)dst, nx, ny, nxp);
    else
        hipLaunchKernelGGL(k_pad<double>, g, b, 0, s, (const double *)src, (double *)dst, nx, ny,
                           nxp);
    return hipGetLastError();
}

}  // namespace lbf
