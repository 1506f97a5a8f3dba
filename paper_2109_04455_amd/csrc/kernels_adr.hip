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
// LBE_ADE, BGK, second-order equilibrium with cs^2 = 1/3; the reaction
// source of Eq. source_lbm acts on a link only when its population heads into
// a catalytic solid node) and Sec.
// "Boundary conditions and flux computation in ADE" (Eq. BC, inlet C_A = 1
// with bounce-back for the other species, outlet C_w = C_b, outflux plane
// two nodes before the right boundary).
#include "adr_device.hpp"
#include "adr_march.hpp"

namespace lbf {
namespace {

using namespace adr;

// 16-byte vectors of V consecutive nodes
template <typename Real, int V, bool NT = false>
__device__ __forceinline__ void vload(const Real *p, Real (&o)[V])
{
    typedef Real nv __attribute__((ext_vector_type(V)));
    const nv v = ld<NT>(reinterpret_cast<const nv *>(p));
#pragma unroll
    for (int j = 0; j < V; ++j) o[j] = v[j];
}

template <typename Real, int V, bool NT = false>
__device__ __forceinline__ void vstore(Real *p, const Real (&o)[V])
{
    typedef Real nv __attribute__((ext_vector_type(V)));
    nv v;
#pragma unroll
    for (int j = 0; j < V; ++j) v[j] = o[j];
    st<NT>(reinterpret_cast<nv *>(p), v);
}

// Vectorised step: each thread owns V consecutive nodes of one row and moves
// every population array with one 16-byte access per array.  The E (W)
// populations pulled from x-1 (x+1) come from the aligned vector of the
// node's own x range plus one scalar element just outside it.  Results are
// identical to k_adr_step node by node.
template <typename Real, typename Acc, int S, bool TRACE, int V, bool NT>
__global__ __launch_bounds__(256) void k_adr_step_vec(AdrArgs<Real> a)
{
    int xv, y;
    tile_coords(a.L, xv, y);
    const int x0 = xv * V;
    if (x0 >= a.nx || y >= a.ny) return;
    const size_t id0 = (size_t)y * a.nxp + x0;
    const size_t P = a.plane;
    unsigned m[V];
    bool any = false, need_own_s = false, need_own_n = false;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        m[j] = a.mask5[id0 + j];
        const bool fl = m[j] != MASK5_SOLID;
        any |= fl;
        need_own_s |= fl && (m[j] & BIT_S);
        need_own_n |= fl && (m[j] & BIT_N);
        need_own_s |= fl && (x0 + j == a.nx - 1);
        need_own_n |= fl && (x0 + j == a.nx - 1);
    }
    if (!any) return;
    Real ux[V], uy[V];
    vload<Real, V>(a.ua + id0, ux);
    vload<Real, V>(a.ua + P + id0, uy);
    const Acc inlet_e = Acc(2) * w5<Acc>(DE) * (Acc(a.cin) - Acc(a.cref));
    Acc h[S][5][V];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const Real *src = a.src + (size_t)s * 5 * P;
        Real own0[V], ownE[V], ownW[V], upN[V], dnS[V], ownN[V] = {}, ownS[V] = {};
        vload<Real, V, NT>(src + id0, own0);
        vload<Real, V, NT>(src + DE * P + id0, ownE);
        vload<Real, V, NT>(src + DW * P + id0, ownW);
        vload<Real, V, NT>(src + DN * P + id0 - a.nxp, upN);
        vload<Real, V, NT>(src + DS * P + id0 + a.nxp, dnS);
        const Real eL = x0 > 0 ? ld<NT>(src + DE * P + id0 - 1) : Real(0);
        const Real wR = x0 + V < a.nx ? ld<NT>(src + DW * P + id0 + V) : Real(0);
        if (need_own_n) vload<Real, V, NT>(src + DN * P + id0, ownN);
        if (need_own_s) vload<Real, V, NT>(src + DS * P + id0, ownS);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int x = x0 + j;
            h[s][0][j] = own0[j];
            if (x == 0)
                h[s][DE][j] = s == 0 ? inlet_e - Acc(ownW[j]) : Acc(ownW[j]);
            else if (m[j] & BIT_W)
                h[s][DE][j] = ownW[j];
            else
                h[s][DE][j] = j == 0 ? eL : ownE[j - 1];
            h[s][DN][j] = (m[j] & BIT_S) ? ownS[j] : upN[j];
            if (x == a.nx - 1) {
                const Acc sum = Acc(own0[j]) + Acc(ownE[j]) + Acc(ownN[j]) + Acc(ownW[j]) + Acc(ownS[j]);
                h[s][DW][j] = Acc(2) * w5<Acc>(DW) * sum - Acc(ownE[j]);
            } else if (m[j] & BIT_E) {
                h[s][DW][j] = ownE[j];
            } else {
                h[s][DW][j] = j == V - 1 ? wR : ownW[j + 1];
            }
            h[s][DS][j] = (m[j] & BIT_N) ? ownN[j] : dnS[j];
        }
    }
    Real out[S][5][V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        Acc hn[S][5];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < 5; ++i) hn[s][i] = h[s][i][j];
        const bool fl = m[j] != MASK5_SOLID;
        if (fl) collide_react<Real, Acc, S, TRACE>(a, id0 + j, m[j], Acc(ux[j]), Acc(uy[j]), hn);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < 5; ++i) out[s][i][j] = fl ? Real(hn[s][i]) : Real(0);
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 5; ++i) vstore<Real, V, NT>(a.dst + (s * 5 + i) * P + id0, out[s][i]);
}

template <typename Real, typename Acc, int S, bool TRACE, bool NT, bool WIDE>
__global__ __launch_bounds__(1024) void k_adr_step(AdrArgs<Real> a)
{
    int x, y;
    tile_coords(a.L, x, y);
    if (x >= a.nx || y >= a.ny) return;
    adr::node_update<Real, Acc, S, TRACE, NT, WIDE>(a, x, y);
}

template <typename Real, typename Acc, int S, bool NT, bool WIDE, bool TRACE>
__global__ __launch_bounds__(64 * (adr::PairTile<Real>::EY + 1))
__attribute__((amdgpu_waves_per_eu(adr::PairTile<Real>::OCC))) void k_adr_step2(AdrArgs<Real> a)
{
    int bx, by;
    tile_of_block(a.L, bx, by);
    adr::pair_update<Real, Acc, S, NT, WIDE, TRACE>(a, bx, by);
}

// Two steps per launch by marching wavefronts (adr_march.hpp): block b holds
// MARCH_WAVES strips side by side in x; strips of odd strip rows march down.
template <int S, bool NT, int H>
__global__ __launch_bounds__(64 * adr::MARCH_WAVES)
__attribute__((amdgpu_waves_per_eu(3))) void k_adr_march(AdrArgs<float> a)
{
    int bx, by;
    tile_of_block(a.L, bx, by);
    const int x0 = (bx * adr::MARCH_WAVES + (int)(threadIdx.x >> 6)) * 64;
    if (x0 >= a.nx) return;  // a whole wavefront past the lattice
    const int y0 = by * H;
    if (by & 1)
        adr::march_strip<S, NT, -1, H>(a, x0, y0);
    else
        adr::march_strip<S, NT, 1, H>(a, x0, y0);
}

// Reaction variant and/or periodic box (FP64 arithmetic, no trace).
template <typename Real, int S, bool NT, int MODE, bool PERIODIC>
__global__ __launch_bounds__(1024) void k_adr_step_ext(AdrArgs<Real> a)
{
    int x, y;
    tile_coords(a.L, x, y);
    if (x >= a.nx || y >= a.ny) return;
    adr::node_update_ext<Real, S, NT, MODE, PERIODIC>(a, x, y);
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
    double p[5];
    eq_factors(double(a.ua[id]), double(a.ua[P + id]), p);
    double h[S][5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        // g_A = w_i c_in (1 + p_i), stored as g_A - w_i cref
        h[0][i] = w5<double>(i) * (a.cin * p[i] + (a.cin - a.cref));
#pragma unroll
        for (int s = 1; s < S; ++s) h[s][i] = 0;
    }
    // first collision with the lattice's reaction rule and neighbour indices
    size_t nb[5];
    if (a.L.periodic) {
        periodic_neighbours(x, y, a.nx, a.ny, a.nxp, nb);
    } else {
        const int off[5] = {0, 1, a.nxp, -1, -a.nxp};
#pragma unroll
        for (int d = 0; d < 5; ++d) nb[d] = id + off[d];
    }
    const double u = double(a.ua[id]), v = double(a.ua[P + id]);
    if (a.L.mode == 1)
        collide_react<Real, double, S, false, 1>(a, id, m, u, v, h, nb);
    else
        collide_react<Real, double, S, false, 0>(a, id, m, u, v, h, nb);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 5; ++i) a.dst[(s * 5 + i) * P + id] = Real(h[s][i]);
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
    double c = 0;
    if (m != MASK5_SOLID) {
        double h[5];
        const double inlet_e = 2.0 * w5<double>(DE) * (a.cin - a.cref);
        if (a.L.periodic) {
            size_t nb[5];
            periodic_neighbours(x, y, a.nx, a.ny, a.nxp, nb);
            pull5_periodic<Real, double, false>(a.src + (size_t)species * 5 * a.plane, a.plane, id,
                                                nb, m, h);
        } else {
            pull5<Real, double, false, true>(a.src + (size_t)species * 5 * a.plane, a.plane, id, x, a.nx,
                                       a.nxp, m, species == 0, inlet_e, h);
        }
        c = (species == 0 ? a.cref : 0.0) + (h[0] + h[1] + h[2] + h[3] + h[4]);
    }
    out[(size_t)y * a.nx + x] = Real(c);
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
    const double inlet_e = 2.0 * w5<double>(DE) * (a.cin - a.cref);
    double h[5];
    pull5<Real, double, false, true>(a.src, a.plane, id, x, a.nx, a.nxp, m, true, inlet_e, h);
    a.trace[2 * t] = Real(a.cref + (h[0] + h[1] + h[2] + h[3] + h[4]));
    double cb = 0;
    if (S == 3) {
        pull5<Real, double, false, true>(a.src + 5 * a.plane, a.plane, id, x, a.nx, a.nxp, m, false,
                                   inlet_e, h);
        cb = h[0] + h[1] + h[2] + h[3] + h[4];
    }
    a.trace[2 * t + 1] = Real(cb);
}

// Total amount of every species after the last step (FP64 sums over the
// fluid nodes; per-block partials, then one block in fixed order).
template <typename Real, int S>
__global__ __launch_bounds__(256) void k_totals(AdrArgs<Real> a, double *partial)
{
    __shared__ double sm[S][256];
    double acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0;
    const size_t n = (size_t)a.nx * a.ny;
    const double inlet_e = 2.0 * w5<double>(DE) * (a.cin - a.cref);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % a.nx), y = (int)(i / a.nx);
        const size_t id = (size_t)y * a.nxp + x;
        const unsigned m = a.mask5[id];
        if (m == MASK5_SOLID) continue;
        size_t nb[5];
        if (a.L.periodic) periodic_neighbours(x, y, a.nx, a.ny, a.nxp, nb);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            double h[5];
            if (a.L.periodic)
                pull5_periodic<Real, double, false>(a.src + (size_t)s * 5 * a.plane, a.plane, id, nb, m, h);
            else
                pull5<Real, double, false, true>(a.src + (size_t)s * 5 * a.plane, a.plane, id, x, a.nx,
                                           a.nxp, m, s == 0, inlet_e, h);
            acc[s] += (s == 0 ? a.cref : 0.0) + (h[0] + h[1] + h[2] + h[3] + h[4]);
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) sm[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
#pragma unroll
            for (int s = 0; s < S; ++s) sm[s][threadIdx.x] += sm[s][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int s = 0; s < S; ++s) partial[(size_t)s * gridDim.x + blockIdx.x] = sm[s][0];
}

// Amount each reaction converts in the step from the state `a.src` streams
// into (Eq. source_lbm summed over the lattice, FP64): partial[q] sums
// A -> B (q = 0) and B -> C (q = 1) per block, fixed reduction order.  The
// concentration of a node is its pulled pre-collision one; link reactions
// take the rate of the catalytic node, the all-populations variant the mean
// rate of the node's catalytic neighbours of the type.
template <typename Real, int S>
__global__ __launch_bounds__(256) void k_production(AdrArgs<Real> a, double *partial)
{
    __shared__ double sm[2][256];
    double acc[2] = {0.0, 0.0};
    const size_t n = (size_t)a.nx * a.ny;
    const double inlet_e = 2.0 * w5<double>(DE) * (a.cin - a.cref);
    const int off[5] = {0, 1, a.nxp, -1, -a.nxp};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % a.nx), y = (int)(i / a.nx);
        const size_t id = (size_t)y * a.nxp + x;
        const unsigned m = a.mask5[id];
        if (m == MASK5_SOLID || !(m & 0xF0u)) continue;
        size_t nb[5];
        if (a.L.periodic) periodic_neighbours(x, y, a.nx, a.ny, a.nxp, nb);
        double c[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            double h[5];
            if (a.L.periodic)
                pull5_periodic<Real, double, false>(a.src + (size_t)s * 5 * a.plane, a.plane, id, nb, m, h);
            else
                pull5<Real, double, false, true>(a.src + (size_t)s * 5 * a.plane, a.plane, id, x, a.nx,
                                                 a.nxp, m, s == 0, inlet_e, h);
            c[s] = (s == 0 ? a.cref : 0.0) + (h[0] + h[1] + h[2] + h[3] + h[4]);
        }
        double ks[2] = {0.0, 0.0};
        int kc[2] = {0, 0};
#pragma unroll
        for (int d = 1; d < 5; ++d) {
            if (!((m >> (3 + d)) & 1u)) continue;
            const size_t sid = a.L.periodic ? nb[d] : id + off[d];
            const int q = a.type[sid] == 2 ? 0 : 1;
            if (q == 1 && S == 2) continue;
            if (a.L.mode == 0) {
                acc[q] += (double)a.kr[sid] * w5<double>(d) * c[q];
            } else {
                ks[q] += (double)a.kr[sid];
                kc[q] += 1;
            }
        }
        if (a.L.mode != 0)
#pragma unroll
            for (int q = 0; q < 2; ++q)
                if (kc[q]) acc[q] += ks[q] / kc[q] * c[q];
    }
    sm[0][threadIdx.x] = acc[0];
    sm[1][threadIdx.x] = acc[1];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            sm[0][threadIdx.x] += sm[0][threadIdx.x + st];
            sm[1][threadIdx.x] += sm[1][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = sm[0][0];
        partial[gridDim.x + blockIdx.x] = sm[1][0];
    }
}

__global__ __launch_bounds__(256) void k_sum_partials(const double *partial, int nblocks, int ns,
                                                      double *out)
{
    __shared__ double sm[256];
    for (int s = 0; s < ns; ++s) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partial[(size_t)s * nblocks + i];
        sm[threadIdx.x] = acc;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[s] = sm[0];
        __syncthreads();
    }
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

template <typename Real, typename Acc, int S, bool TRACE, bool NT>
void step_launch(const AdrArgs<Real> &a, hipStream_t s)
{
    constexpr int V = 16 / sizeof(Real);
    if (a.L.vec)
        hipLaunchKernelGGL((k_adr_step_vec<Real, Acc, S, TRACE, V, NT>), a.L.grid(), a.L.block(), 0,
                           s, a);
    else if (a.L.wide)
        hipLaunchKernelGGL((k_adr_step<Real, Acc, S, TRACE, NT, true>), a.L.grid(), a.L.block(), 0,
                           s, a);
    else
        hipLaunchKernelGGL((k_adr_step<Real, Acc, S, TRACE, NT, false>), a.L.grid(), a.L.block(),
                           0, s, a);
}

template <typename Real, typename Acc, int S>
void step_launch_nt(bool trace, bool nt, const AdrArgs<Real> &a, hipStream_t s)
{
    if (trace)
        nt ? step_launch<Real, Acc, S, true, true>(a, s) : step_launch<Real, Acc, S, true, false>(a, s);
    else
        nt ? step_launch<Real, Acc, S, false, true>(a, s) : step_launch<Real, Acc, S, false, false>(a, s);
}

// FP64 storage always computes in FP64; FP32 storage computes in FP64 unless
// the launch asks for FP32 arithmetic.
template <typename Real, int S, bool NT>
void ext_launch(const AdrArgs<Real> &a, hipStream_t s)
{
    const dim3 g = a.L.grid(), b = a.L.block();
    if (a.L.mode == 1) {
        if (a.L.periodic)
            hipLaunchKernelGGL((k_adr_step_ext<Real, S, NT, 1, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_adr_step_ext<Real, S, NT, 1, false>), g, b, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_adr_step_ext<Real, S, NT, 0, true>), g, b, 0, s, a);
    }
}

template <typename Real>
hipError_t step_dispatch(int ns, bool trace, const AdrArgs<Real> &a, hipStream_t s)
{
    const bool nt = a.L.nontemporal;
    if (a.L.mode != 0 || a.L.periodic) {
        if (ns == 2)
            nt ? ext_launch<Real, 2, true>(a, s) : ext_launch<Real, 2, false>(a, s);
        else
            nt ? ext_launch<Real, 3, true>(a, s) : ext_launch<Real, 3, false>(a, s);
        return hipGetLastError();
    }
    const bool f32math = sizeof(Real) == 4 && a.L.fp32_math;
    if (ns == 2) {
        if (f32math)
            step_launch_nt<Real, float, 2>(trace, nt, a, s);
        else
            step_launch_nt<Real, double, 2>(trace, nt, a, s);
    } else {
        if (f32math)
            step_launch_nt<Real, float, 3>(trace, nt, a, s);
        else
            step_launch_nt<Real, double, 3>(trace, nt, a, s);
    }
    return hipGetLastError();
}

template <typename Real, typename Acc, int S>
void pair_launch(const AdrArgs<Real> &a, hipStream_t s)
{
    const dim3 b(64 * (adr::PairTile<Real>::EY + 1));
    const dim3 g = a.L.grid();
    const int sel = (a.L.nontemporal ? 1 : 0) | (a.L.wide ? 2 : 0) | (a.trace || a.trace2 ? 4 : 0);
    switch (sel) {
    case 0: hipLaunchKernelGGL((k_adr_step2<Real, Acc, S, false, false, false>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_adr_step2<Real, Acc, S, true, false, false>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_adr_step2<Real, Acc, S, false, true, false>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_adr_step2<Real, Acc, S, true, true, false>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_adr_step2<Real, Acc, S, false, false, true>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_adr_step2<Real, Acc, S, true, false, true>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_adr_step2<Real, Acc, S, false, true, true>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_adr_step2<Real, Acc, S, true, true, true>), g, b, 0, s, a); break;
    }
}

template <typename Real>
hipError_t pair_dispatch(int ns, const AdrArgs<Real> &a, hipStream_t s)
{
    if (a.L.tx != adr::PairTile<Real>::TX || a.L.ty != adr::PairTile<Real>::TY) return hipErrorInvalidValue;
    if constexpr (sizeof(Real) == 4) {
        if (a.L.fp32_math) {
            ns == 2 ? pair_launch<Real, float, 2>(a, s) : pair_launch<Real, float, 3>(a, s);
            return hipGetLastError();
        }
    }
    ns == 2 ? pair_launch<Real, double, 2>(a, s) : pair_launch<Real, double, 3>(a, s);
    return hipGetLastError();
}

}  // namespace

Launch march_launch(const Launch &base, int nx, int ny, int h)
{
    Launch L = base;
    L.tx = 64 * adr::MARCH_WAVES;
    L.ty = h;  // strip height; blocks are 64 * MARCH_WAVES threads
    const int strips = (nx + 63) / 64;
    L.gx = (strips + adr::MARCH_WAVES - 1) / adr::MARCH_WAVES;
    L.gy = (ny + h - 1) / h;
    L.vec = false;
    return L;
}

hipError_t launch_adr_march(int ns, const AdrArgs<float> &a, hipStream_t s)
{
    if (a.L.tx != 64 * adr::MARCH_WAVES || a.L.wide || a.L.fp32_math || a.L.mode != 0 ||
        a.L.periodic || a.trace || a.trace2)
        return hipErrorInvalidValue;
    const dim3 g = a.L.grid(), b(64 * adr::MARCH_WAVES);
    const bool nt = a.L.nontemporal;
#define LBF_MARCH(H)                                                                   \
    if (a.L.ty == H) {                                                                 \
        if (ns == 2 && nt)                                                             \
            hipLaunchKernelGGL((k_adr_march<2, true, H>), g, b, 0, s, a);              \
        else if (ns == 2)                                                              \
            hipLaunchKernelGGL((k_adr_march<2, false, H>), g, b, 0, s, a);             \
        else if (nt)                                                                   \
            hipLaunchKernelGGL((k_adr_march<3, true, H>), g, b, 0, s, a);              \
        else                                                                           \
            hipLaunchKernelGGL((k_adr_march<3, false, H>), g, b, 0, s, a);             \
        return hipGetLastError();                                                      \
    }
    LBF_MARCH(22)
#undef LBF_MARCH
    return hipErrorInvalidValue;
    return hipGetLastError();
}

void pair_tile(int real_bytes, int &tx, int &ty)
{
    tx = real_bytes == 4 ? adr::PairTile<float>::TX : adr::PairTile<double>::TX;
    ty = real_bytes == 4 ? adr::PairTile<float>::TY : adr::PairTile<double>::TY;
}

hipError_t launch_adr_pair(int real_bytes, int ns, const AdrArgs<float> &af,
                           const AdrArgs<double> &ad, hipStream_t s)
{
    return real_bytes == 4 ? pair_dispatch(ns, af, s) : pair_dispatch(ns, ad, s);
}

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

hipError_t launch_totals(int real_bytes, int ns, const AdrArgs<float> &af, const AdrArgs<double> &ad,
                         double *partial, int nblocks, double *out, hipStream_t s)
{
    const dim3 g(nblocks), b(256);
    if (real_bytes == 4) {
        if (ns == 2) hipLaunchKernelGGL((k_totals<float, 2>), g, b, 0, s, af, partial);
        else hipLaunchKernelGGL((k_totals<float, 3>), g, b, 0, s, af, partial);
    } else {
        if (ns == 2) hipLaunchKernelGGL((k_totals<double, 2>), g, b, 0, s, ad, partial);
        else hipLaunchKernelGGL((k_totals<double, 3>), g, b, 0, s, ad, partial);
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partial, nblocks, ns, out);
    return hipGetLastError();
}

hipError_t launch_production(int real_bytes, int ns, const AdrArgs<float> &af,
                             const AdrArgs<double> &ad, double *partial, int nblocks, double *out,
                             hipStream_t s)
{
    const dim3 g(nblocks), b(256);
    if (real_bytes == 4) {
        if (ns == 2) hipLaunchKernelGGL((k_production<float, 2>), g, b, 0, s, af, partial);
        else hipLaunchKernelGGL((k_production<float, 3>), g, b, 0, s, af, partial);
    } else {
        if (ns == 2) hipLaunchKernelGGL((k_production<double, 2>), g, b, 0, s, ad, partial);
        else hipLaunchKernelGGL((k_production<double, 3>), g, b, 0, s, ad, partial);
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partial, nblocks, 2, out);
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
