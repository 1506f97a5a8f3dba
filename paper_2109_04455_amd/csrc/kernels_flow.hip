// D2Q9 BGK flow kernels: one fused pull-stream / collide step per launch.
//
// Storage: populations after collision, shifted by their weights
// (h_i = f_i - w_i, so that rho = 1 + sum h_i keeps FP32 precision), as a
// structure of arrays [9][ny][nxp].  A step gathers h_i(x - c_i) (half-way
// bounce-back at solid sources, Zou-He at the inlet x = 0 and outlet
// x = nx-1), forms rho and u, relaxes to the second-order equilibrium with
// omega = 1/tau_f and writes the result in place of the node's own slots of
// the destination lattice.
//
// Paper: Sec. "Lattice-Boltzmann for the Navier-Stokes equation" (Eq. LBE;
// bounce-back at the fibre surfaces).  The paper drives a periodic 3D box by
// a body force; this 2D channel is driven by a parabolic velocity inlet
// (Zou & He, 1997) instead.
#include "flow_device.hpp"

namespace lbf {
namespace {

using namespace flow;

template <typename Real, typename Acc, bool WRITE_U, bool NT, bool WIDE>
__global__ __launch_bounds__(1024) void k_flow_step(FlowArgs<Real> a)
{
    int x, y;
    tile_coords(a.L, x, y);
    if (x >= a.nx || y >= a.ny) return;
    flow::node_update<Real, Acc, WRITE_U, NT, WIDE>(a, x, y);
}

// Two rows per thread (FP64 arithmetic): the launch covers ceil(ny / 2)
// tile rows, thread row y taking lattice rows 2y and 2y + 1.
template <typename Real, typename Acc, bool WRITE_U, bool NT, bool WIDE>
__global__ __launch_bounds__(1024) void k_flow_step2r(FlowArgs<Real> a)
{
    int x, y;
    tile_coords(a.L, x, y);
    y *= 2;
    if (x >= a.nx || y >= a.ny) return;
    flow::node_update2<Real, Acc, WRITE_U, NT, WIDE>(a, x, y);
}

// Two steps per launch (FP64 arithmetic), one block per tile of the
// two-step tiling (flow::pair_update).
template <typename Real, bool WRITE_U, bool NT, bool WIDE>
__global__ __launch_bounds__(64 * (FlowPairTile<Real>::EY + 1))
__attribute__((amdgpu_waves_per_eu(FlowPairTile<Real>::OCC))) void k_flow_pair(FlowArgs<Real> a)
{
    int bx, by;
    tile_of_block(a.L, bx, by);
    flow::pair_update<Real, double, WRITE_U, NT, WIDE>(a, bx, by);
}

template <typename Real>
hipError_t flow_pair_launch(bool write_u, const FlowArgs<Real> &a, hipStream_t s)
{
    using T = FlowPairTile<Real>;
    if (a.L.tx != T::TX || a.L.ty != T::TY || a.L.fp32_math) return hipErrorInvalidValue;
    const dim3 g = a.L.grid(), b(64 * (T::EY + 1));
    const int sel = (write_u ? 1 : 0) | (a.L.nontemporal ? 2 : 0) | (a.L.wide ? 4 : 0);
    switch (sel) {
    case 0: hipLaunchKernelGGL((k_flow_pair<Real, false, false, false>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_flow_pair<Real, true, false, false>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_flow_pair<Real, false, true, false>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_flow_pair<Real, true, true, false>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_flow_pair<Real, false, false, true>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_flow_pair<Real, true, false, true>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_flow_pair<Real, false, true, true>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_flow_pair<Real, true, true, true>), g, b, 0, s, a); break;
    }
    return hipGetLastError();
}

// Lattices below this many nodes (launch-bound: a few blocks per step) keep
// one row per thread.
constexpr long FLOW_TWO_ROWS_MIN_NODES = 1L << 18;

template <typename Real, typename Acc, bool WIDE>
void flow_launch_w(bool write_u, const FlowArgs<Real> &a, hipStream_t s)
{
    if (sizeof(Acc) == 8 && (long)a.nx * a.ny >= FLOW_TWO_ROWS_MIN_NODES) {
        FlowArgs<Real> a2 = a;
        a2.L.gy = ((a.ny + 1) / 2 + a.L.ty - 1) / a.L.ty;
        const dim3 g = a2.L.grid(), b = a2.L.block();
        if (a.L.nontemporal) {
            if (write_u) hipLaunchKernelGGL((k_flow_step2r<Real, Acc, true, true, WIDE>), g, b, 0, s, a2);
            else hipLaunchKernelGGL((k_flow_step2r<Real, Acc, false, true, WIDE>), g, b, 0, s, a2);
        } else {
            if (write_u) hipLaunchKernelGGL((k_flow_step2r<Real, Acc, true, false, WIDE>), g, b, 0, s, a2);
            else hipLaunchKernelGGL((k_flow_step2r<Real, Acc, false, false, WIDE>), g, b, 0, s, a2);
        }
        return;
    }
    const dim3 g = a.L.grid(), b = a.L.block();
    if (a.L.nontemporal) {
        if (write_u)
            hipLaunchKernelGGL((k_flow_step<Real, Acc, true, true, WIDE>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_flow_step<Real, Acc, false, true, WIDE>), g, b, 0, s, a);
    } else {
        if (write_u)
            hipLaunchKernelGGL((k_flow_step<Real, Acc, true, false, WIDE>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_flow_step<Real, Acc, false, false, WIDE>), g, b, 0, s, a);
    }
}

template <typename Real, typename Acc>
void flow_launch_acc(bool write_u, const FlowArgs<Real> &a, hipStream_t s)
{
    if (a.L.wide)
        flow_launch_w<Real, Acc, true>(write_u, a, s);
    else
        flow_launch_w<Real, Acc, false>(write_u, a, s);
}

template <typename Real>
void flow_launch(bool write_u, const FlowArgs<Real> &a, hipStream_t s)
{
    if (sizeof(Real) == 4 && a.L.fp32_math)
        flow_launch_acc<Real, float>(write_u, a, s);
    else
        flow_launch_acc<Real, double>(write_u, a, s);
}

// Initial state f = f_eq(1, (u_in(y), 0)), then one collision (the stored
// state is always post-collision).
template <typename Real>
__global__ __launch_bounds__(1024) void k_flow_init(FlowArgs<Real> a)
{
    int x, y;
    tile_coords(a.L, x, y);
    if (x >= a.nx || y >= a.ny) return;
    const size_t id = (size_t)y * a.nxp + x;
    const size_t P = a.plane;
    const unsigned m = a.mask9[id];
    if (m & MASK9_SOLID) {
        a.u[id] = 0;
        a.u[P + id] = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) a.dst[i * P + id] = 0;
        return;
    }
    const double ux = inlet_u<double>(y, a.ny, a.u0);
    double h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double cu = double(CX[i]) * ux;
        h[i] = wgt<double>(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * ux * ux);
    }
    double u, v;
    collide(h, a.omega, u, v);
    a.u[id] = Real(u);
    a.u[P + id] = Real(v);
#pragma unroll
    for (int i = 0; i < 9; ++i) a.dst[i * P + id] = Real(h[i]);
}

// max |u - u_prev| over fluid nodes (both components); copies u -> u_prev.
// Non-finite velocities give +inf.  Per-block maxima, then one block.
template <typename Real>
__global__ __launch_bounds__(256) void k_du_max(const Real *u, Real *uprev, const uint16_t *mask9,
                                                size_t plane, double *partial)
{
    __shared__ double sm[256];
    double mx = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * plane;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t id = i < plane ? i : i - plane;
        if (mask9[id] & MASK9_SOLID) continue;
        const double a = (double)u[i], b = (double)uprev[i];
        double d = fabs(a - b);
        if (!isfinite(a)) d = INFINITY;
        mx = fmax(mx, d);
        uprev[i] = u[i];
    }
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_max_partials(const double *partial, int n, double *out)
{
    __shared__ double sm[256];
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, partial[i]);
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

}  // namespace

hipError_t launch_flow_init(int real_bytes, const FlowArgs<float> &af, const FlowArgs<double> &ad,
                            hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_flow_init<float>, af.L.grid(), af.L.block(), 0, s, af);
    else
        hipLaunchKernelGGL(k_flow_init<double>, ad.L.grid(), ad.L.block(), 0, s, ad);
    return hipGetLastError();
}

hipError_t launch_flow_step(int real_bytes, bool write_u, const FlowArgs<float> &af,
                            const FlowArgs<double> &ad, hipStream_t s)
{
    if (real_bytes == 4)
        flow_launch(write_u, af, s);
    else
        flow_launch(write_u, ad, s);
    return hipGetLastError();
}

hipError_t launch_flow_pair(int real_bytes, bool write_u, const FlowArgs<float> &af,
                            const FlowArgs<double> &ad, hipStream_t s)
{
    return real_bytes == 4 ? flow_pair_launch(write_u, af, s) : flow_pair_launch(write_u, ad, s);
}

hipError_t launch_du_max(int real_bytes, const void *u, void *uprev, const uint16_t *mask9,
                         size_t plane, double *partial, int nblocks, double *out, hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_du_max<float>, dim3(nblocks), dim3(256), 0, s, (const float *)u,
                           (float *)uprev, mask9, plane, partial);
    else
        hipLaunchKernelGGL(k_du_max<double>, dim3(nblocks), dim3(256), 0, s, (const double *)u,
                           (double *)uprev, mask9, plane, partial);
    hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(256), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_du_max_partials(const double *partial, int n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(256), 0, s, partial, n, out);
    return hipGetLastError();
}

}  // namespace lbf
