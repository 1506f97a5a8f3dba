// 3D kernels: D3Q19 flow with a body force (Guo forcing) in a box periodic in
// every direction, D3Q7 stream-collide-react with inlet/outlet in x and
// periodic y, z, and their set-up kernels and reductions.  One thread per
// node; the launch tiles (x, row) with row = z * ny + y.
#include "lbf3d_internal.hpp"

namespace lbf {
namespace d3 {
namespace {

template <typename T>
__device__ __forceinline__ T w19(int i)
{
    return i == 0 ? T(1) / T(3) : (i < 7 ? T(1) / T(18) : T(1) / T(36));
}

template <typename T>
__device__ __forceinline__ T w7(int i)
{
    return i == 0 ? T(0.25) : T(0.125);
}

// ----------------------------------------------------------------- masks ----
__global__ void k_masks3(const uint8_t *type_in, uint8_t *type_pad, uint16_t *mask7,
                         uint32_t *mask19, Geo g, int nspecies)
{
    const size_t n = g.plane;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % g.nxp), row = (int)(i / g.nxp);
        if (x >= g.nx) {
            type_pad[i] = 1;
            mask7[i] = MASK7_SOLID;
            mask19[i] = MASK19_SOLID;
            continue;
        }
        const int y = row % g.ny, z = row / g.ny;
        const uint8_t t = type_in[(size_t)row * g.nx + x];
        type_pad[i] = t;
        if (t != 0) {
            mask7[i] = MASK7_SOLID;
            mask19[i] = MASK19_SOLID;
            continue;
        }
        uint32_t m19 = 0;
        unsigned m7 = 0;
        for (int d = 1; d < 19; ++d) {
            int xx = x + CX[d];
            xx = xx < 0 ? xx + g.nx : (xx >= g.nx ? xx - g.nx : xx);
            const int r = row_of(g, y, z, CY[d], CZ[d]);
            if (type_in[(size_t)r * g.nx + xx] != 0) m19 |= 1u << (d - 1);
            if (d < 7) {
                // D3Q7 shares the first six D3Q19 directions; x is not periodic
                const int x7 = x + CX[d];
                if (x7 < 0 || x7 >= g.nx) continue;
                const uint8_t tn = type_in[(size_t)r * g.nx + x7];
                if (tn != 0) m7 |= 1u << (d - 1);
                if (tn == 2 || (tn == 3 && nspecies == 3)) m7 |= 1u << (d + 5);
            }
        }
        mask7[i] = (uint16_t)m7;
        mask19[i] = m19;
    }
}

template <typename Real>
__global__ void k_copy_rates3(const double *k_in, const uint8_t *type_pad, Real *kr, Geo g)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.plane;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % g.nxp), row = (int)(i / g.nxp);
        const uint8_t t = type_pad[i];
        kr[i] = (x < g.nx && (t == 2 || t == 3)) ? Real(k_in[(size_t)row * g.nx + x]) : Real(0);
    }
}

// ------------------------------------------------------------------ flow ----
// Collide (BGK + Guo force along x) the shifted populations h = f - w in
// place; u is the physical velocity (j + F/2)/rho.  Deviation form as in 2D:
// 1/rho = 1 + d with d = -drho/(1 + drho), rho X = X + drho X.
template <typename T>
__device__ __forceinline__ void collide19(T (&h)[19], T omega, T fx, T (&u)[3])
{
    T drho = h[0];
    T j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        drho += h[i];
        if (CX[i]) j[0] += CX[i] > 0 ? h[i] : -h[i];
        if (CY[i]) j[1] += CY[i] > 0 ? h[i] : -h[i];
        if (CZ[i]) j[2] += CZ[i] > 0 ? h[i] : -h[i];
    }
    const T d = -drho / (T(1) + drho);
    const T jx = j[0] + T(0.5) * fx;
    u[0] = jx + jx * d;
    u[1] = j[1] + j[1] * d;
    u[2] = j[2] + j[2] * d;
    const T uu = T(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const T fs = (T(1) - T(0.5) * omega) * fx;  // force prefactor
    {
        const T x0 = -uu;
        const T eq = w19<T>(0) * (drho + (x0 + drho * x0));
        h[0] -= omega * (h[0] - eq);
        h[0] += w19<T>(0) * fs * (T(-3) * u[0]);
    }
#pragma unroll
    for (int p = 1; p < 19; p += 2) {
        const T cu = T(CX[p]) * u[0] + T(CY[p]) * u[1] + T(CZ[p]) * u[2];
        const T w = w19<T>(p);
        const T xe = T(4.5) * cu * cu - uu;
        const T xo = T(3) * cu;
        const T even = drho + (xe + drho * xe);
        const T odd = xo + drho * xo;
        // Guo source w (1 - omega/2) [3 (c_x - u_x) + 9 (c.u) c_x] F
        const T se = T(9) * cu * T(CX[p]) - T(3) * u[0];
        const T so = T(3) * T(CX[p]);
        h[p] -= omega * (h[p] - w * (even + odd));
        h[p + 1] -= omega * (h[p + 1] - w * (even - odd));
        h[p] += w * fs * (se + so);
        h[p + 1] += w * fs * (se - so);
    }
}

// Populations are read and written at 64-bit byte offsets from the lattice
// base (32-bit buffer offsets, which pay off in 2D, measured slower here).
template <typename Real, typename Acc, bool WRITE_U, bool NT>
__global__ __launch_bounds__(1024) void k_flow_step3(FlowArgs3<Real> a)
{
    using Off = size_t;
    constexpr Off QB = SEG * sizeof(Real);  // bytes between populations q and q + 1
    int x, row;
    tile_coords(a.L, x, row);
    const Geo &g = a.g;
    if (x >= g.nx || row >= g.ny * g.nz) return;
    const Off id = (Off)row * (Off)g.nxp + (Off)x;
    const uint32_t m = a.mask19[id];
    if (m & MASK19_SOLID) return;
    const int y = row % g.ny, z = row / g.ny;
    const Off PB = (Off)g.plane * sizeof(Real);
    const PopBlock<Real, NT, true> in(a.src, 19 * PB), out(a.dst, 19 * PB);
    const Off own = seg_off<19, Real>(id);
    Acc h[19];
    h[0] = Acc(in.load(own));
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const int o = opp19(i);
        Off src;
        if ((m >> (o - 1)) & 1u) {
            src = own + (Off)o * QB;  // half-way bounce-back
        } else {
            int sx = x - CX[i];
            sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
            const Off sid = (Off)row_of(g, y, z, -CY[i], -CZ[i]) * (Off)g.nxp + (Off)sx;
            src = seg_off<19, Real>(sid) + (Off)i * QB;
        }
        h[i] = Acc(in.load(src));
    }
    Acc u[3];
    collide19(h, Acc(a.omega), Acc(a.fx), u);
    if (WRITE_U) {
        a.u[id] = Real(u[0]);
        a.u[g.plane + id] = Real(u[1]);
        a.u[2 * g.plane + id] = Real(u[2]);
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) out.store(own + (Off)i * QB, Real(h[i]));
}

template <typename Real>
__global__ __launch_bounds__(1024) void k_flow_init3(FlowArgs3<Real> a)
{
    int x, row;
    tile_coords(a.L, x, row);
    const Geo &g = a.g;
    if (x >= g.nx || row >= g.ny * g.nz) return;
    const size_t id = (size_t)row * g.nxp + x;
    const size_t P = g.plane;
    if (a.mask19[id] & MASK19_SOLID) {
        for (int i = 0; i < 19; ++i) a.dst[pidx<19>(id, i)] = Real(0);
        for (int c = 0; c < 3; ++c) a.u[(size_t)c * P + id] = Real(0);
        return;
    }
    double h[19];
    for (int i = 0; i < 19; ++i) h[i] = 0.0;
    double u[3];
    collide19(h, a.omega, a.fx, u);
    for (int c = 0; c < 3; ++c) a.u[(size_t)c * P + id] = Real(u[c]);
    for (int i = 0; i < 19; ++i) a.dst[pidx<19>(id, i)] = Real(h[i]);
}

// max |u - uprev| and max |u| over fluid nodes (per-block partials), then
// uprev = u.
template <typename Real>
__global__ __launch_bounds__(256) void k_du_max3(const Real *u, Real *uprev, const uint32_t *mask19,
                                                 size_t plane, double *partial)
{
    __shared__ double sd[256], su[256];
    double md = 0.0, mu = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane;
         i += (size_t)gridDim.x * blockDim.x) {
        if (mask19[i] & MASK19_SOLID) continue;
        double du2 = 0.0, u2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double a = (double)u[c * plane + i], b = (double)uprev[c * plane + i];
            du2 += (a - b) * (a - b);
            u2 += a * a;
            uprev[c * plane + i] = u[c * plane + i];
        }
        double dd = sqrt(du2);
        if (!isfinite(u2)) dd = INFINITY;
        md = fmax(md, dd);
        mu = fmax(mu, sqrt(u2));
    }
    sd[threadIdx.x] = md;
    su[threadIdx.x] = mu;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
            su[threadIdx.x] = fmax(su[threadIdx.x], su[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sd[0];
        partial[2 * blockIdx.x + 1] = su[0];
    }
}

__global__ __launch_bounds__(256) void k_max2(const double *partial, int n, double *out2)
{
    __shared__ double sd[256], su[256];
    double md = 0.0, mu = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        md = fmax(md, partial[2 * i]);
        mu = fmax(mu, partial[2 * i + 1]);
    }
    sd[threadIdx.x] = md;
    su[threadIdx.x] = mu;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
            su[threadIdx.x] = fmax(su[threadIdx.x], su[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = sd[0];
        out2[1] = su[0];
    }
}

template <typename Real>
__global__ void k_handoff3(const Real *u, Real *ua, const uint16_t *mask7, size_t plane,
                           double scale)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane;
         i += (size_t)gridDim.x * blockDim.x) {
        const bool fl = mask7[i] != MASK7_SOLID;
        for (int c = 0; c < 3; ++c)
            ua[c * plane + i] = fl ? Real(scale * (double)u[c * plane + i]) : Real(0);
    }
}

// [3][plane] <-> [3][nz][ny][nx]
template <typename Real>
__global__ void k_unpad3(const Real *src, Real *dst, Geo g)
{
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t c = i / n, r = i % n;
        const size_t row = r / g.nx, x = r % g.nx;
        dst[i] = src[c * g.plane + row * g.nxp + x];
    }
}

template <typename Real>
__global__ void k_pad3(const Real *src, Real *dst, const uint8_t *type_pad, Geo g)
{
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * g.plane;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t c = i / g.plane, r = i % g.plane;
        const size_t row = r / g.nxp, x = r % g.nxp;
        dst[i] = (x < (size_t)g.nx && type_pad[r] == 0) ? src[c * n + row * g.nx + x] : Real(0);
    }
}

// ------------------------------------------------------------------- ADR ----
// Gather the pre-collision shifted populations of one species (populations
// q0 .. q0+6 of a lattice of NQ populations) at node (x, row) from the
// previous post-collision lattice.  Directions 1..6 = +x, -x, +y, -y, +z, -z;
// so[d]: byte offset (seg_off) of neighbour x + c_d, so[0] of the node itself.
template <typename Real, typename Acc, int NQ, typename Blk, typename Off>
__device__ __forceinline__ void pull7(const Blk &lat, int q0, const Off (&so)[7], int x, int nx,
                                      unsigned m, bool species_a, Acc inlet_e, Acc (&h)[7])
{
    constexpr Off QB = SEG * sizeof(Real);
    auto at = [&](int node, int d) { return Acc(lat.load(so[node] + (Off)(q0 + d) * QB)); };
    h[0] = at(0, 0);
    // +x arrives from x - 1
    if (x == 0)
        h[1] = species_a ? inlet_e - at(0, 2) : at(0, 2);
    else if (m & 2u)
        h[1] = at(0, 2);
    else
        h[1] = at(2, 1);
    // -x arrives from x + 1
    if (x == nx - 1) {
        Acc sum = Acc(0);
#pragma unroll
        for (int j = 0; j < 7; ++j) sum += at(0, j);
        h[2] = Acc(2) * w7<Acc>(2) * sum - at(0, 1);
    } else if (m & 1u) {
        h[2] = at(0, 1);
    } else {
        h[2] = at(1, 2);
    }
    // +-y, +-z: periodic; bounce-back at solid neighbours
#pragma unroll
    for (int d = 3; d < 7; ++d) {
        const int o = d & 1 ? d + 1 : d - 1;
        h[d] = (m >> (o - 1)) & 1u ? at(0, o) : at(o, d);
    }
}

// The same for all S species of the node at once (species s at populations
// 7s .. 7s+6): the sources are chosen by offset and all 7 S loads are issued
// before any is converted to Acc.  A branch per direction with the
// conversion inside made each species wait for its loads in turn.  Outlet
// nodes read their own populations for the outlet rule afterwards.  Same
// results as pull7 per species.
template <typename Real, typename Acc, int S, typename Blk, typename Off>
__device__ __forceinline__ void pull7S(const Blk &lat, const Off (&so)[7], int x, int nx,
                                       unsigned m, Acc inlet_e, Acc (&h)[S][7])
{
    constexpr Off QB = SEG * sizeof(Real);
    const bool in = x == 0, out = x == nx - 1;
    Off src[7];
    src[0] = so[0];
    src[1] = (in || (m & 2u)) ? so[0] + 2 * QB : so[2] + 1 * QB;   // +x from x - 1
    src[2] = (out || (m & 1u)) ? so[0] + 1 * QB : so[1] + 2 * QB;  // -x from x + 1
#pragma unroll
    for (int d = 3; d < 7; ++d) {
        const int o = d & 1 ? d + 1 : d - 1;
        src[d] = ((m >> (o - 1)) & 1u) ? so[0] + (Off)o * QB : so[o] + (Off)d * QB;
    }
    Real r[S][7];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int d = 0; d < 7; ++d) r[s][d] = lat.load(src[d] + (Off)(7 * s) * QB);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int d = 0; d < 7; ++d) h[s][d] = Acc(r[s][d]);
    if (in) h[0][1] = inlet_e - h[0][1];
    if (out) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            // h[s][2] holds the node's own +x population here
            Acc sum = Acc(0);
            sum += h[s][0];
            sum += h[s][2];
#pragma unroll
            for (int j = 2; j < 7; ++j) sum += Acc(lat.load(so[0] + (Off)(7 * s + j) * QB));
            h[s][2] = Acc(2) * w7<Acc>(2) * sum - h[s][2];
        }
    }
}

// Indices of the six neighbours x + c_d (x unwrapped: only used in range).
template <typename Idx>
__device__ __forceinline__ void neighbours7(const Geo &g, int x, int y, int z, Idx (&nb)[7])
{
    const Idx r = (Idx)(z * g.ny + y) * (Idx)g.nxp;
    nb[0] = r + x;
    nb[1] = r + x + 1;
    nb[2] = r + x - 1;
    nb[3] = (Idx)row_of(g, y, z, 1, 0) * (Idx)g.nxp + x;
    nb[4] = (Idx)row_of(g, y, z, -1, 0) * (Idx)g.nxp + x;
    nb[5] = (Idx)row_of(g, y, z, 0, 1) * (Idx)g.nxp + x;
    nb[6] = (Idx)row_of(g, y, z, 0, -1) * (Idx)g.nxp + x;
}

// Byte offsets (seg_off) of a node's neighbours in a lattice of NQ populations.
template <int NQ, typename Real, typename Idx>
__device__ __forceinline__ void neighbour_offsets(const Idx (&nb)[7], Idx (&so)[7])
{
#pragma unroll
    for (int d = 0; d < 7; ++d) so[d] = seg_off<NQ, Real>(nb[d]);
}

// Collide (second-order equilibrium, cs^2 = 1/4) and react one node in place.
template <typename Real, typename Acc, int S, typename Idx>
__device__ __forceinline__ void collide_react7(const AdrArgs3<Real> &a, unsigned m,
                                               const Idx (&nb)[7], Acc u, Acc v, Acc w,
                                               Acc (&h)[S][7])
{
    const Acc uu = Acc(2) * (u * u + v * v + w * w);
    Acc p[7];
    p[0] = -uu;
    const Acc cu[3] = {u, v, w};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const Acc e = Acc(8) * cu[q] * cu[q] - uu;
        p[1 + 2 * q] = e + Acc(4) * cu[q];
        p[2 + 2 * q] = e - Acc(4) * cu[q];
    }
    Acc c[S];
    const Acc omega = Acc(a.omega);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        Acc delta = h[s][0];
#pragma unroll
        for (int i = 1; i < 7; ++i) delta += h[s][i];
        const Acc cref = s == 0 ? Acc(a.cref) : Acc(0);
        c[s] = cref + delta;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            const Acc wi = w7<Acc>(i);
            const Acc target = wi * p[i] * cref + wi * (Acc(1) + p[i]) * delta;
            h[s][i] -= omega * (h[s][i] - target);
        }
    }
    if (m & 0xFC0u) {
        // Eq. source_lbm at the links into catalytic nodes
#pragma unroll
        for (int d = 1; d < 7; ++d) {
            if (!((m >> (d + 5)) & 1u)) continue;
            const Idx sid = nb[d];
            const Acc k = Acc(a.kr[sid]);
            if (a.type[sid] == 2) {
                const Acc r = k * w7<Acc>(d) * c[0];
                h[0][d] -= r;
                h[1][d] += r;
            } else if (S == 3) {
                const Acc r = k * w7<Acc>(d) * c[1];
                h[1][d] -= r;
                h[S - 1][d] += r;
            }
        }
    }
}

template <typename Real, typename Acc, int S, bool NT>
__global__ __launch_bounds__(1024) void k_adr_step3(AdrArgs3<Real> a)
{
    using Off = size_t;
    constexpr int NQ = 7 * S;
    constexpr Off QB = SEG * sizeof(Real);
    int x, row;
    tile_coords(a.L, x, row);
    const Geo &g = a.g;
    if (x >= g.nx || row >= g.ny * g.nz) return;
    const Off id = (Off)row * (Off)g.nxp + (Off)x;
    const unsigned m = a.mask7[id];
    if (m == MASK7_SOLID) return;
    const int y = row % g.ny, z = row / g.ny;
    const Off PB = (Off)g.plane * sizeof(Real);
    Off nb[7], so[7];
    neighbours7(g, x, y, z, nb);
    neighbour_offsets<NQ, Real>(nb, so);
    const PopBlock<Real, NT, true> in(a.src, NQ * PB), out(a.dst, NQ * PB);
    const PopBlock<Real, false, true> vel(a.ua, 3 * PB);
    const Acc inlet_e = Acc(2) * w7<Acc>(1) * (Acc(a.cin) - Acc(a.cref));
    Acc h[S][7];
    pull7S<Real, Acc, S>(in, so, x, g.nx, m, inlet_e, h);
    const Off ob = id * (Off)sizeof(Real);
    collide_react7<Real, Acc, S>(a, m, nb, Acc(vel.load(ob)), Acc(vel.load(ob + PB)),
                                 Acc(vel.load(ob + 2 * PB)), h);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < 7; ++i) out.store(so[0] + (Off)(7 * s + i) * QB, Real(h[s][i]));
}

// A at equilibrium with C = c_in, B = C = 0, then the first collision.
template <typename Real, int S>
__global__ __launch_bounds__(1024) void k_adr_init3(AdrArgs3<Real> a)
{
    int x, row;
    tile_coords(a.L, x, row);
    const Geo &g = a.g;
    if (x >= g.nx || row >= g.ny * g.nz) return;
    const size_t id = (size_t)row * g.nxp + x;
    const size_t P = g.plane;
    const unsigned m = a.mask7[id];
    if (m == MASK7_SOLID) {
        for (int s = 0; s < S; ++s)
            for (int i = 0; i < 7; ++i) a.dst[pidx<7 * S>(id, 7 * s + i)] = Real(0);
        return;
    }
    const int y = row % g.ny, z = row / g.ny;
    size_t nb[7];
    neighbours7(g, x, y, z, nb);
    const double u = a.ua[id], v = a.ua[P + id], w = a.ua[2 * P + id];
    const double uu = 2.0 * (u * u + v * v + w * w);
    const double cu[7] = {0.0, u, -u, v, -v, w, -w};
    double h[S][7];
    for (int i = 0; i < 7; ++i) {
        const double p = 4.0 * cu[i] + 8.0 * cu[i] * cu[i] - uu;
        // g_A = w_i c_in (1 + p_i), stored as g_A - w_i cref
        h[0][i] = w7<double>(i) * (a.cin * p + (a.cin - a.cref));
        for (int s = 1; s < S; ++s) h[s][i] = 0.0;
    }
    collide_react7<Real, double, S>(a, m, nb, u, v, w, h);
    for (int s = 0; s < S; ++s)
        for (int i = 0; i < 7; ++i) a.dst[pidx<7 * S>(id, 7 * s + i)] = Real(h[s][i]);
}

// Outlet fluxes through the face xf + 1/2 and the inlet flux of A, from the
// previous post-collision lattice (one block, fixed summation order):
// N_s = sum over rows of post_{+x}(xf) - post_{-x}(xf + 1) where both nodes
// are fluid; inflow = sum over fluid rows at x = 0 of
// 2 w (c_in - cref) - 2 post_{-x,A}(0).
template <typename Real, int S>
__global__ __launch_bounds__(1024) void k_flux3(AdrArgs3<Real> a, int xf, double *out4)
{
    __shared__ double sm[4][1024];
    const Geo &g = a.g;
    double acc[4] = {0, 0, 0, 0};
    const int rows = g.ny * g.nz;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const size_t i0 = (size_t)r * g.nxp;
        if (a.mask7[i0 + xf] != MASK7_SOLID && a.mask7[i0 + xf + 1] != MASK7_SOLID)
            for (int s = 0; s < S; ++s)
                acc[s] += (double)a.src[pidx<7 * S>(i0 + xf, 7 * s + 1)] -
                          (double)a.src[pidx<7 * S>(i0 + xf + 1, 7 * s + 2)];
        if (a.mask7[i0] != MASK7_SOLID)
            acc[3] += 2.0 * 0.125 * (a.cin - a.cref) - 2.0 * (double)a.src[pidx<7 * S>(i0, 2)];
    }
    for (int s = 0; s < 4; ++s) sm[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int s = 0; s < 4; ++s) sm[s][threadIdx.x] += sm[s][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int s = 0; s < 4; ++s) out4[s] = s < S || s == 3 ? sm[s][0] : 0.0;
}

// Pre-collision concentration of one species after the last step.
template <typename Real, int S>
__global__ __launch_bounds__(1024) void k_conc3(AdrArgs3<Real> a, int species, Real *out)
{
    int x, row;
    tile_coords(a.L, x, row);
    const Geo &g = a.g;
    if (x >= g.nx || row >= g.ny * g.nz) return;
    const size_t id = (size_t)row * g.nxp + x;
    const unsigned m = a.mask7[id];
    double c = 0.0;
    if (m != MASK7_SOLID) {
        const int y = row % g.ny, z = row / g.ny;
        size_t nb[7], so[7];
        neighbours7(g, x, y, z, nb);
        neighbour_offsets<7 * S, Real>(nb, so);
        const PopBlock<Real, false, true> lat(a.src, 0);
        double h[7];
        const double inlet_e = 2.0 * 0.125 * (a.cin - a.cref);
        pull7<Real, double, 7 * S>(lat, 7 * species, so, x, g.nx, m, species == 0, inlet_e, h);
        c = species == 0 ? a.cref : 0.0;
        for (int i = 0; i < 7; ++i) c += h[i];
    }
    out[(size_t)row * g.nx + x] = Real(c);
}

template <typename Real, int S>
__global__ __launch_bounds__(256) void k_totals3(AdrArgs3<Real> a, double *partial)
{
    __shared__ double sm[S][256];
    const Geo &g = a.g;
    double acc[S];
    for (int s = 0; s < S; ++s) acc[s] = 0.0;
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    const double inlet_e = 2.0 * 0.125 * (a.cin - a.cref);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % g.nx), row = (int)(i / g.nx);
        const size_t id = (size_t)row * g.nxp + x;
        const unsigned m = a.mask7[id];
        if (m == MASK7_SOLID) continue;
        const int y = row % g.ny, z = row / g.ny;
        size_t nb[7], so[7];
        neighbours7(g, x, y, z, nb);
        neighbour_offsets<7 * S, Real>(nb, so);
        const PopBlock<Real, false, true> lat(a.src, 0);
        for (int s = 0; s < S; ++s) {
            double h[7];
            pull7<Real, double, 7 * S>(lat, 7 * s, so, x, g.nx, m, s == 0, inlet_e, h);
            double c = s == 0 ? a.cref : 0.0;
            for (int j = 0; j < 7; ++j) c += h[j];
            acc[s] += c;
        }
    }
    for (int s = 0; s < S; ++s) sm[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int s = 0; s < S; ++s) sm[s][threadIdx.x] += sm[s][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int s = 0; s < S; ++s) partial[(size_t)s * gridDim.x + blockIdx.x] = sm[s][0];
}

__global__ __launch_bounds__(256) void k_sum_partials3(const double *partial, int nblocks, int ns,
                                                       double *out)
{
    __shared__ double sm[256];
    for (int s = 0; s < ns; ++s) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < nblocks; i += blockDim.x) acc += partial[(size_t)s * nblocks + i];
        sm[threadIdx.x] = acc;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[s] = sm[0];
        __syncthreads();
    }
}

}  // namespace

// ------------------------------------------------------------ launchers ----
hipError_t launch_masks3(const uint8_t *type_in, uint8_t *type_pad, uint16_t *mask7,
                         uint32_t *mask19, const Geo &g, int nspecies, hipStream_t s)
{
    hipLaunchKernelGGL(k_masks3, dim3(4096), dim3(256), 0, s, type_in, type_pad, mask7, mask19, g,
                       nspecies);
    return hipGetLastError();
}

hipError_t launch_copy_rates3(const double *k_in, const uint8_t *type_pad, void *kr,
                              int real_bytes, const Geo &g, hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_copy_rates3<float>, dim3(4096), dim3(256), 0, s, k_in, type_pad,
                           (float *)kr, g);
    else
        hipLaunchKernelGGL(k_copy_rates3<double>, dim3(4096), dim3(256), 0, s, k_in, type_pad,
                           (double *)kr, g);
    return hipGetLastError();
}

hipError_t launch_flow_init3(int real_bytes, const FlowArgs3<float> &af,
                             const FlowArgs3<double> &ad, hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_flow_init3<float>, af.L.grid(), af.L.block(), 0, s, af);
    else
        hipLaunchKernelGGL(k_flow_init3<double>, ad.L.grid(), ad.L.block(), 0, s, ad);
    return hipGetLastError();
}

template <typename Real, typename Acc>
static void flow_launch3(bool write_u, const FlowArgs3<Real> &a, hipStream_t s)
{
    const dim3 gr = a.L.grid(), b = a.L.block();
    if (a.L.nontemporal) {
        if (write_u) hipLaunchKernelGGL((k_flow_step3<Real, Acc, true, true>), gr, b, 0, s, a);
        else hipLaunchKernelGGL((k_flow_step3<Real, Acc, false, true>), gr, b, 0, s, a);
    } else {
        if (write_u) hipLaunchKernelGGL((k_flow_step3<Real, Acc, true, false>), gr, b, 0, s, a);
        else hipLaunchKernelGGL((k_flow_step3<Real, Acc, false, false>), gr, b, 0, s, a);
    }
}

hipError_t launch_flow_step3(int real_bytes, bool write_u, const FlowArgs3<float> &af,
                             const FlowArgs3<double> &ad, hipStream_t s)
{
    if (real_bytes == 4) {
        if (af.L.fp32_math) flow_launch3<float, float>(write_u, af, s);
        else flow_launch3<float, double>(write_u, af, s);
    } else {
        flow_launch3<double, double>(write_u, ad, s);
    }
    return hipGetLastError();
}

hipError_t launch_du_max3(int real_bytes, const void *u, void *uprev, const uint32_t *mask19,
                          size_t plane, double *partial, int nblocks, double *out2, hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_du_max3<float>, dim3(nblocks), dim3(256), 0, s, (const float *)u,
                           (float *)uprev, mask19, plane, partial);
    else
        hipLaunchKernelGGL(k_du_max3<double>, dim3(nblocks), dim3(256), 0, s, (const double *)u,
                           (double *)uprev, mask19, plane, partial);
    hipLaunchKernelGGL(k_max2, dim3(1), dim3(256), 0, s, partial, nblocks, out2);
    return hipGetLastError();
}

hipError_t launch_velocity_handoff3(int real_bytes, const void *u, void *ua, const uint16_t *mask7,
                                    size_t plane, double scale, hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_handoff3<float>, dim3(4096), dim3(256), 0, s, (const float *)u,
                           (float *)ua, mask7, plane, scale);
    else
        hipLaunchKernelGGL(k_handoff3<double>, dim3(4096), dim3(256), 0, s, (const double *)u,
                           (double *)ua, mask7, plane, scale);
    return hipGetLastError();
}

hipError_t launch_unpad3(int real_bytes, const void *src, void *dst, const Geo &g, hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_unpad3<float>, dim3(4096), dim3(256), 0, s, (const float *)src,
                           (float *)dst, g);
    else
        hipLaunchKernelGGL(k_unpad3<double>, dim3(4096), dim3(256), 0, s, (const double *)src,
                           (double *)dst, g);
    return hipGetLastError();
}

hipError_t launch_pad3(int real_bytes, const void *src, void *dst, const uint8_t *type_pad,
                       const Geo &g, hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_pad3<float>, dim3(4096), dim3(256), 0, s, (const float *)src,
                           (float *)dst, type_pad, g);
    else
        hipLaunchKernelGGL(k_pad3<double>, dim3(4096), dim3(256), 0, s, (const double *)src,
                           (double *)dst, type_pad, g);
    return hipGetLastError();
}

hipError_t launch_adr_init3(int real_bytes, int ns, const AdrArgs3<float> &af,
                            const AdrArgs3<double> &ad, hipStream_t s)
{
    if (real_bytes == 4) {
        if (ns == 2) hipLaunchKernelGGL((k_adr_init3<float, 2>), af.L.grid(), af.L.block(), 0, s, af);
        else hipLaunchKernelGGL((k_adr_init3<float, 3>), af.L.grid(), af.L.block(), 0, s, af);
    } else {
        if (ns == 2) hipLaunchKernelGGL((k_adr_init3<double, 2>), ad.L.grid(), ad.L.block(), 0, s, ad);
        else hipLaunchKernelGGL((k_adr_init3<double, 3>), ad.L.grid(), ad.L.block(), 0, s, ad);
    }
    return hipGetLastError();
}

template <typename Real, typename Acc, int S>
static void adr_launch3(const AdrArgs3<Real> &a, hipStream_t s)
{
    if (a.L.nontemporal)
        hipLaunchKernelGGL((k_adr_step3<Real, Acc, S, true>), a.L.grid(), a.L.block(), 0, s, a);
    else
        hipLaunchKernelGGL((k_adr_step3<Real, Acc, S, false>), a.L.grid(), a.L.block(), 0, s, a);
}

hipError_t launch_adr_step3(int real_bytes, int ns, const AdrArgs3<float> &af,
                            const AdrArgs3<double> &ad, hipStream_t s)
{
    if (real_bytes == 4) {
        if (af.L.fp32_math) {
            if (ns == 2) adr_launch3<float, float, 2>(af, s);
            else adr_launch3<float, float, 3>(af, s);
        } else {
            if (ns == 2) adr_launch3<float, double, 2>(af, s);
            else adr_launch3<float, double, 3>(af, s);
        }
    } else {
        if (ns == 2) adr_launch3<double, double, 2>(ad, s);
        else adr_launch3<double, double, 3>(ad, s);
    }
    return hipGetLastError();
}

hipError_t launch_flux3(int real_bytes, int ns, const AdrArgs3<float> &af,
                        const AdrArgs3<double> &ad, int xf, double *out4, hipStream_t s)
{
    if (real_bytes == 4) {
        if (ns == 2) hipLaunchKernelGGL((k_flux3<float, 2>), dim3(1), dim3(1024), 0, s, af, xf, out4);
        else hipLaunchKernelGGL((k_flux3<float, 3>), dim3(1), dim3(1024), 0, s, af, xf, out4);
    } else {
        if (ns == 2) hipLaunchKernelGGL((k_flux3<double, 2>), dim3(1), dim3(1024), 0, s, ad, xf, out4);
        else hipLaunchKernelGGL((k_flux3<double, 3>), dim3(1), dim3(1024), 0, s, ad, xf, out4);
    }
    return hipGetLastError();
}

hipError_t launch_concentration3(int real_bytes, int ns, int species, const AdrArgs3<float> &af,
                                 const AdrArgs3<double> &ad, void *out, hipStream_t s)
{
    if (real_bytes == 4) {
        if (ns == 2) hipLaunchKernelGGL((k_conc3<float, 2>), af.L.grid(), af.L.block(), 0, s, af, species, (float *)out);
        else hipLaunchKernelGGL((k_conc3<float, 3>), af.L.grid(), af.L.block(), 0, s, af, species, (float *)out);
    } else {
        if (ns == 2) hipLaunchKernelGGL((k_conc3<double, 2>), ad.L.grid(), ad.L.block(), 0, s, ad, species, (double *)out);
        else hipLaunchKernelGGL((k_conc3<double, 3>), ad.L.grid(), ad.L.block(), 0, s, ad, species, (double *)out);
    }
    return hipGetLastError();
}

hipError_t launch_totals3(int real_bytes, int ns, const AdrArgs3<float> &af,
                          const AdrArgs3<double> &ad, double *partial, int nblocks, double *out,
                          hipStream_t s)
{
    const dim3 gr(nblocks), b(256);
    if (real_bytes == 4) {
        if (ns == 2) hipLaunchKernelGGL((k_totals3<float, 2>), gr, b, 0, s, af, partial);
        else hipLaunchKernelGGL((k_totals3<float, 3>), gr, b, 0, s, af, partial);
    } else {
        if (ns == 2) hipLaunchKernelGGL((k_totals3<double, 2>), gr, b, 0, s, ad, partial);
        else hipLaunchKernelGGL((k_totals3<double, 3>), gr, b, 0, s, ad, partial);
    }
    hipLaunchKernelGGL(k_sum_partials3, dim3(1), dim3(256), 0, s, partial, nblocks, ns, out);
    return hipGetLastError();
}

}  // namespace d3
}  // namespace lbf
