// GPU random-walk particle tracker (include/lbf_rw.h): one thread per
// particle, particles held as structure-of-arrays, the reservoir refilled
// every step and the particles that left dropped by an order-preserving
// stream compaction every few steps (skipped by the move in between),
// crossing counts in 64-bit integer atomics.  A step is a fixed chain of
// kernels whose sizes live on the device, so blocks of steps are captured as
// HIP graphs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "lbf_rw.h"

namespace {

constexpr uint64_t GAMMA = 0x9e3779b97f4a7c15ULL;  // splitmix64 increment
constexpr uint64_t ID_INSERT = 1ULL << 62;
constexpr uint64_t ID_COUNT = 1ULL << 63;
constexpr int SCAN_BLOCKS = 1024;  // blocks of every scan pass (fixed: sizes are on the device)
constexpr int SCAN_THREADS = 256;
// the arrays are compacted at the start of every graph block and every
// compact_every steps inside one (nx / 8, between 1 and 64: a step inserts
// about 1/nx of the particles the domain holds, so the slots of those that
// left in between stay within an eighth of them); in between, particles that
// left stay in place (skipped by the move)
constexpr long COMPACT_MAX = 64;
constexpr double BUF_LO = -1.5, BUF_HI = -0.5;  // reservoir strip

__device__ __forceinline__ uint64_t mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// draw d of step t of particle id: output 8 t + d + 1 of splitmix64 started
// from seed ^ mix(id), as a double in [0, 1)
__device__ __forceinline__ double draw(uint64_t seed, uint64_t id, uint64_t t, unsigned d)
{
    const uint64_t state = seed ^ mix(id);
    const uint64_t n = 8 * t + d + 1;
    return (double)(mix(state + n * GAMMA) >> 11) * (1.0 / 9007199254740992.0);
}

struct Field {
    int nx, ny, ns, wall_mode;
    const uint8_t *type;
    const double2 *uv;   // (ux, uy) of each cell, one 16-byte load
    const uint64_t *nb;  // [ny + 6][nx + 6] windows of types, of cells x, y in [-3, n + 3)
    const double *k;
    double vs;      // velocity scale
    double dt, len, zone, rate_w;
    uint64_t seed;
};

__device__ __forceinline__ int cell_of(double p) { return (int)floor(p + 0.5); }

__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Type of cell (x, y) read from the lattice: rows outside are solid (1),
// columns outside fluid (0).
__device__ __forceinline__ int type_read(const Field &f, int x, int y)
{
    if (y < 0 || y >= f.ny) return 1;
    if (x < 0 || x >= f.nx) return 0;
    return f.type[(size_t)y * f.nx + x];
}

// The types of the 5 x 5 cells around a particle's cell (ox, oy), from one
// 64-bit word (2 bits per cell, outside the lattice as type_read).  Words
// exist for ox in [-3, nx + 3) and oy in [-3, ny + 3); beyond, every cell of
// the window lies outside the lattice on that side, so the word of the
// nearest stored cell is the same.  A step shorter than one cell per axis
// lands within one cell of (ox, oy), so its interpolation corners, reflection
// tests, landing cell and that cell's neighbours all lie in the window.
struct Window {
    uint64_t w;
    int ox, oy;
};

__device__ __forceinline__ Window window_at(const Field &f, int ox, int oy)
{
    Window v;
    v.ox = ox;
    v.oy = oy;
    const int wx = ox < -3 ? -3 : (ox > f.nx + 2 ? f.nx + 2 : ox);
    const int wy = oy < -3 ? -3 : (oy > f.ny + 2 ? f.ny + 2 : oy);
    v.w = f.nb[(size_t)(wy + 3) * (f.nx + 6) + (wx + 3)];
    return v;
}

// cell (x, y) within two cells of (ox, oy) in each axis
__device__ __forceinline__ int win_type(const Window &v, int x, int y)
{
    return (int)(v.w >> (2 * (5 * (y - v.oy + 2) + x - v.ox + 2))) & 3;
}

// Cell types for the rest of a step: from the window (steps shorter than a
// cell per axis) or read from the lattice.
struct WinTypes {
    const Window &v;
    __device__ __forceinline__ int operator()(int x, int y) const { return win_type(v, x, y); }
};
struct ReadTypes {
    const Field &f;
    __device__ __forceinline__ int operator()(int x, int y) const { return type_read(f, x, y); }
};

// Bilinear interpolation of the two velocity components at (px, py); in
// wall_mode 1 a solid corner takes minus the mean of its fluid neighbours
// along the cell edges (or minus the diagonal fluid corner), so the
// interpolant is zero on the half-way wall.  Corner classification is shared
// by both components.
__device__ void interp2(const Field &f, const Window &wv, double px, double py, double &uo,
                        double &vo)
{
    const int x0 = (int)floor(px), y0 = (int)floor(py);
    const double fx = px - x0, fy = py - y0;
    double a[2][2], b[2][2];
    bool sol[2][2];
    // the velocities are read at clamped (in-range) cells, all together;
    // solid corners then take 0
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int cx = x0 + i, cy = y0 + j;
            const double2 q = f.uv[(size_t)clampi(cy, f.ny - 1) * f.nx + clampi(cx, f.nx - 1)];
            sol[j][i] = win_type(wv, cx, cy) != 0;
            a[j][i] = sol[j][i] ? 0.0 : q.x;
            b[j][i] = sol[j][i] ? 0.0 : q.y;
        }
    if (f.wall_mode == 1) {
        double wa[2][2], wb[2][2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                wa[j][i] = a[j][i];
                wb[j][i] = b[j][i];
                if (!sol[j][i]) continue;
                double sa = 0.0, sb = 0.0;
                int n = 0;
                if (!sol[j][1 - i]) { sa -= a[j][1 - i]; sb -= b[j][1 - i]; ++n; }
                if (!sol[1 - j][i]) { sa -= a[1 - j][i]; sb -= b[1 - j][i]; ++n; }
                if (n == 0 && !sol[1 - j][1 - i]) { sa -= a[1 - j][1 - i]; sb -= b[1 - j][1 - i]; n = 1; }
                wa[j][i] = n ? sa / n : 0.0;
                wb[j][i] = n ? sb / n : 0.0;
            }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[j][i] = wa[j][i];
                b[j][i] = wb[j][i];
            }
    }
    const double c00 = (1 - fx) * (1 - fy), c01 = fx * (1 - fy), c10 = (1 - fx) * fy, c11 = fx * fy;
    uo = c00 * a[0][0] + c01 * a[0][1] + c10 * a[1][0] + c11 * a[1][1];
    vo = c00 * b[0][0] + c01 * b[0][1] + c10 * b[1][0] + c11 * b[1][1];
}

// Specular reflection of the move (px, py) -> (qx, qy) at the faces of solid
// cells; a move that would still end in a solid cell is cancelled.
template <typename Types>
__device__ __forceinline__ void reflect(const Types &type, double px, double py, double &qx,
                                        double &qy)
{
    const int ox = cell_of(px), oy = cell_of(py);
    const int nxc = cell_of(qx), nyc = cell_of(qy);
    if (type(nxc, nyc) == 0) return;
    bool done = false;
    if (nxc != ox && type(nxc, oy) != 0) {
        qx = 2.0 * (nxc > ox ? ox + 0.5 : ox - 0.5) - qx;
        done = true;
    }
    if (nyc != oy && type(ox, nyc) != 0) {
        qy = 2.0 * (nyc > oy ? oy + 0.5 : oy - 0.5) - qy;
        done = true;
    }
    if (!done) {
        qx = 2.0 * (nxc > ox ? ox + 0.5 : ox - 0.5) - qx;
        qy = 2.0 * (nyc > oy ? oy + 0.5 : oy - 0.5) - qy;
    }
    if (type(cell_of(qx), cell_of(qy)) != 0) {
        qx = px;
        qy = py;
    }
}

// The rest of a step after the move to (x1, y1): reflection, the inlet rule
// for B and C, the crossing of x = plane and the reaction; returns the
// crossing.
template <typename Types>
__device__ __forceinline__ int finish(const Field &f, const Types &type, uint64_t id, uint64_t t,
                                      double buf_hi, double plane, double x0, double y0,
                                      double &x1, double &y1, uint8_t &s)
{
    reflect(type, x0, y0, x1, y1);
    if (x1 < buf_hi && x0 >= buf_hi && s != 0) x1 = 2.0 * buf_hi - x1;  // B, C at the inlet
    const int ds = (x0 < plane && x1 >= plane) ? 1 : ((x0 >= plane && x1 < plane) ? -1 : 0);
    const int cx = cell_of(x1), cy = cell_of(y1);
    if (cx >= 0 && cx < f.nx && cy >= 0 && cy < f.ny && type(cx, cy) == 0) {
        const int DX[4] = {1, 0, -1, 0}, DY[4] = {0, 1, 0, -1};
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const int sx = cx + DX[d], sy = cy + DY[d];
            if (sx < 0 || sx >= f.nx || sy < 0 || sy >= f.ny) continue;
            const int tn = type(sx, sy);
            const int src = tn == 2 ? 0 : (tn == 3 && f.ns == 3 ? 1 : -1);
            if (src != s) continue;
            const double dist = d == 0 ? cx + 0.5 - x1 : d == 1 ? cy + 0.5 - y1
                              : d == 2 ? x1 - (cx - 0.5) : y1 - (cy - 0.5);
            if (dist >= f.zone) continue;
            const double p = f.k[(size_t)sy * f.nx + sx] * f.rate_w * f.dt / f.zone;
            if (draw(f.seed, id, t, 1 + d) < p) {
                s = (uint8_t)(src + 1);
                break;
            }
        }
    }
    return ds;
}

// One step of one particle; returns the signed crossing of x = plane.
__device__ int move(const Field &f, uint64_t id, uint64_t t, double buf_hi, double plane,
                    double &x, double &y, uint8_t &s)
{
    const double x0 = x, y0 = y;
    const int ox = cell_of(x0), oy = cell_of(y0);
    // one load gives every cell type the step needs (in all but steps longer
    // than a cell); it and the corner velocities are the step's gathers
    const Window wv = window_at(f, ox, oy);
    double u, v;
    interp2(f, wv, x0, y0, u, v);
    u *= f.vs;
    v *= f.vs;
    double sn, cs;
    sincos(2.0 * M_PI * draw(f.seed, id, t, 0), &sn, &cs);
    double x1 = x0 + u * f.dt + f.len * cs;
    double y1 = y0 + v * f.dt + f.len * sn;
    const int lx = cell_of(x1) - ox, ly = cell_of(y1) - oy;
    int ds;
    if (lx >= -1 && lx <= 1 && ly >= -1 && ly <= 1)
        ds = finish(f, WinTypes{wv}, id, t, buf_hi, plane, x0, y0, x1, y1, s);
    else
        ds = finish(f, ReadTypes{f}, id, t, buf_hi, plane, x0, y0, x1, y1, s);
    x = x1;
    y = y1;
    return ds;
}

struct Parts {
    double *x, *y;
    uint8_t *sp;
    uint64_t *id;
};

// Scalars kept on the device (so that a step needs no host round trip).
struct Scalars {
    long long n_cur;     // particles in the current arrays
    long long n_alive;   // this step's insertion point (survivors of a compaction)
    long long t;         // this step's number
    long long t_next;    // the next step's number
    long long cross[3];  // signed crossings while measuring
    long long n_held;    // particles moved by the last step
    int overflow;        // capacity was hit
};

// ---- order-preserving chunked scans ----------------------------------------
// Block b owns items [b*chunk, (b+1)*chunk) (chunk a multiple of the block
// size) and walks them in tiles of SCAN_THREADS consecutive items, thread j
// taking item j of each tile, so every access of a wavefront is coalesced.
// Inside a tile the rank of an item comes from a wavefront ballot plus the
// counts of the lower wavefronts; block totals are scanned by one block.

__device__ __forceinline__ void chunk_bounds(long long n, long long &b0, long long &b1)
{
    long long chunk = (n + SCAN_BLOCKS - 1) / SCAN_BLOCKS;
    chunk = (chunk + SCAN_THREADS - 1) / SCAN_THREADS * SCAN_THREADS;
    b0 = min(n, (long long)blockIdx.x * chunk);
    b1 = min(n, b0 + chunk);
}

// rank of this thread's predicate among the set predicates of the tile
// (lower threads first); *tile_total receives the tile's count
__device__ __forceinline__ int tile_rank(bool pred, int *tile_total)
{
    __shared__ int wsum[SCAN_THREADS / 64];
    const unsigned long long m = __ballot(pred);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int in_wave = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int below = 0, total = 0;
#pragma unroll
    for (int w = 0; w < SCAN_THREADS / 64; ++w) {
        below += w < wave ? wsum[w] : 0;
        total += wsum[w];
    }
    __syncthreads();
    *tile_total = total;
    return below + in_wave;
}

__device__ long long block_sum(long long v)
{
    __shared__ long long sm[SCAN_THREADS];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = SCAN_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    const long long r = sm[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ bool alive(double x, int nx) { return x >= BUF_HI && x < nx - 0.5; }

// pass 1 of the compaction: survivors per block
__global__ __launch_bounds__(SCAN_THREADS) void k_count_alive(Parts p, const Scalars *sc, int nx,
                                                               long long *block_total)
{
    long long b0, b1;
    chunk_bounds(sc->n_cur, b0, b1);
    long long c = 0;
    for (long long i = b0 + threadIdx.x; i < b1; i += SCAN_THREADS) c += alive(p.x[i], nx);
    const long long total = block_sum(c);
    if (threadIdx.x == 0) block_total[blockIdx.x] = total;
}

// scan of the block totals (one block of SCAN_BLOCKS threads)
__global__ __launch_bounds__(SCAN_BLOCKS) void k_scan_top(const long long *block_total,
                                                          long long *block_off, long long *total_out)
{
    __shared__ long long sm[SCAN_BLOCKS];
    const long long v = block_total[threadIdx.x];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCKS; off <<= 1) {
        const long long a = threadIdx.x >= (unsigned)off ? sm[threadIdx.x - off] : 0;
        __syncthreads();
        sm[threadIdx.x] += a;
        __syncthreads();
    }
    block_off[threadIdx.x] = sm[threadIdx.x] - v;
    if (threadIdx.x == SCAN_BLOCKS - 1) *total_out = sm[SCAN_BLOCKS - 1];
}

// pass 3: scatter the survivors, order preserved
__global__ __launch_bounds__(SCAN_THREADS) void k_compact(Parts src, Parts dst, const Scalars *sc,
                                                           int nx, const long long *block_off)
{
    long long b0, b1;
    chunk_bounds(sc->n_cur, b0, b1);
    long long base = block_off[blockIdx.x];
    for (long long t = b0; t < b1; t += SCAN_THREADS) {
        const long long i = t + threadIdx.x;
        const double x = i < b1 ? src.x[i] : 0.0;
        const bool a = i < b1 && alive(x, nx);
        int tile_total;
        const int r = tile_rank(a, &tile_total);
        if (a) {
            const long long o = base + r;
            dst.x[o] = x;
            dst.y[o] = src.y[i];
            dst.sp[o] = src.sp[i];
            dst.id[o] = src.id[i];
        }
        base += tile_total;
    }
}

// reservoir refill: buf_count new A particles after the survivors
__global__ void k_insert(Parts dst, Scalars *sc, long long buf_count, long long capacity,
                         uint64_t seed, double ylo, double yhi)
{
    const long long n0 = sc->n_alive;
    const long long t = sc->t;
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < buf_count;
         j += (long long)gridDim.x * blockDim.x) {
        const long long o = n0 + j;
        if (o >= capacity) {
            sc->overflow = 1;
            continue;
        }
        const uint64_t id = ID_INSERT + ((uint64_t)t << 24) + (uint64_t)j;
        dst.x[o] = BUF_LO + (BUF_HI - BUF_LO) * draw(seed, id, 0, 6);
        dst.y[o] = ylo + (yhi - ylo) * draw(seed, id, 0, 7);
        dst.sp[o] = 0;
        dst.id[o] = id;
    }
}

// Start of a step: its number, its insertion point (a step without
// compaction appends after every particle of the arrays, the ones that left
// since the last compaction included) and its particle count with the
// reservoir refill.
__global__ void k_step_begin(Scalars *sc, long long buf_count, long long capacity, int lazy)
{
    if (lazy) sc->n_alive = sc->n_cur;
    const long long n = sc->n_alive + buf_count;
    sc->n_cur = n < capacity ? n : capacity;
    sc->n_held = 0;
    sc->t = sc->t_next;
    sc->t_next = sc->t + 1;
}

// move every particle; crossing counts reduced per block, then one atomic
// per block and species.  Particles below this step's insertion point
// (n_alive) that are no longer alive left the domain since the last
// compaction and stay where they are until the next one removes them; the
// particles moved are counted (n_held).  At most 96 VGPRs (five wavefronts
// per SIMD, two registers spilled) hide more of the gathers' latency than 101
// VGPRs and four wavefronts; six wavefronts spill 17 and run slower.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_move(Field f, Parts p, Scalars *sc, double plane,
                                              int measure)
{
    __shared__ long long cnt[4];
    if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
    __syncthreads();
    const long long n = sc->n_cur, first_new = sc->n_alive;
    const uint64_t t = (uint64_t)sc->t;
    int c[3] = {0, 0, 0};
    int moved = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double x = p.x[i], y = p.y[i];
        if (i < first_new && !alive(x, f.nx)) continue;
        uint8_t s = p.sp[i];
        const uint8_t s0 = s;
        const int ds = move(f, p.id[i], t, BUF_HI, plane, x, y, s);
        c[s0] += ds;
        ++moved;
        p.x[i] = x;
        p.y[i] = y;
        p.sp[i] = s;
    }
    if (moved) atomicAdd((unsigned long long *)&cnt[3], (unsigned long long)moved);
    if (measure)
        for (int s = 0; s < 3; ++s)
            if (c[s]) atomicAdd((unsigned long long *)&cnt[s], (unsigned long long)(long long)c[s]);
    __syncthreads();
    if (measure && threadIdx.x < 3 && cnt[threadIdx.x])
        atomicAdd((unsigned long long *)&sc->cross[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
    if (threadIdx.x == 3 && cnt[3])
        atomicAdd((unsigned long long *)&sc->n_held, (unsigned long long)cnt[3]);
}


// Per cell: the velocity pair; per cell (ox, oy) of [-3, nx + 3) x
// [-3, ny + 3): the types of the 5 x 5 cells around it (bits
// 2 (5 (dy + 2) + dx + 2)), outside the lattice as type_read.
__global__ void k_pack_fields(Field f, const double *ux, const double *uy, double2 *uv, uint64_t *nb)
{
    const long long n = (long long)f.nx * f.ny, nw = (long long)(f.nx + 6) * (f.ny + 6);
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nw;
         c += (long long)gridDim.x * blockDim.x) {
        if (c < n) uv[c] = make_double2(ux[c], uy[c]);
        const int ox = (int)(c % (f.nx + 6)) - 3, oy = (int)(c / (f.nx + 6)) - 3;
        uint64_t w = 0;
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx)
                w |= (uint64_t)type_read(f, ox + dx, oy + dy) << (2 * (5 * (dy + 2) + dx + 2));
        nb[c] = w;
    }
}

// ---- initial fill ------------------------------------------------------------
__global__ void k_fill_count(Field f, double density, int *counts)
{
    const long long n = (long long)f.nx * f.ny;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x)
        counts[c] = f.type[c] == 0 ? (int)floor(density + draw(f.seed, ID_COUNT + (uint64_t)c, 0, 0)) : 0;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_fill_sum(const int *counts, long long ncell,
                                                            long long *block_total)
{
    long long b0, b1;
    chunk_bounds(ncell, b0, b1);
    long long c = 0;
    for (long long i = b0 + threadIdx.x; i < b1; i += SCAN_THREADS) c += counts[i];
    const long long total = block_sum(c);
    if (threadIdx.x == 0) block_total[blockIdx.x] = total;
}

// exclusive scan over the block (LDS); *total receives the block sum
__device__ long long block_exscan(long long v, long long *total)
{
    __shared__ long long sm[SCAN_THREADS];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        const long long a = threadIdx.x >= (unsigned)off ? sm[threadIdx.x - off] : 0;
        __syncthreads();
        sm[threadIdx.x] += a;
        __syncthreads();
    }
    const long long incl = sm[threadIdx.x];
    *total = sm[SCAN_THREADS - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_fill_place(Field f, const int *counts,
                                                              const long long *block_off, Parts dst,
                                                              long long capacity, Scalars *sc)
{
    const long long ncell = (long long)f.nx * f.ny;
    long long b0, b1;
    chunk_bounds(ncell, b0, b1);
    long long base = block_off[blockIdx.x];
    for (long long t = b0; t < b1; t += SCAN_THREADS) {
        const long long cidx = t + threadIdx.x;
        const int n = cidx < b1 ? counts[cidx] : 0;
        long long tile_total;
        long long o = base + block_exscan(n, &tile_total);
        const int cx = (int)(cidx % f.nx), cy = (int)(cidx / f.nx);
        for (int j = 0; j < n; ++j, ++o) {
            if (o >= capacity) {
                sc->overflow = 1;
                continue;
            }
            const uint64_t id = (uint64_t)cidx * 256 + (uint64_t)j;
            dst.x[o] = cx - 0.5 + draw(f.seed, id, 0, 6);
            dst.y[o] = cy - 0.5 + draw(f.seed, id, 0, 7);
            dst.sp[o] = 0;
            dst.id[o] = id;
        }
        base += tile_total;
    }
}

__global__ void k_fill_finish(Scalars *sc, const long long *total, long long capacity)
{
    const long long n = *total;
    sc->n_cur = n < capacity ? n : capacity;
    sc->n_alive = 0;
    sc->t = sc->t_next = 0;
    sc->cross[0] = sc->cross[1] = sc->cross[2] = 0;
    sc->n_held = sc->n_cur;
}

__global__ void k_walk(Field f, long long np, const uint64_t *ids, double *x, double *y,
                       uint8_t *sp, long long t0, long long steps)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (long long)gridDim.x * blockDim.x) {
        double px = x[i], py = y[i];
        uint8_t s = sp[i];
        for (long long t = t0; t < t0 + steps; ++t)
            (void)move(f, ids[i], (uint64_t)t, BUF_HI, f.nx + 10.0, px, py, s);
        x[i] = px;
        y[i] = py;
        sp[i] = s;
    }
}

}  // namespace

struct lbf_rw_s {
    lbf_rw_params p{};
    bool valid = false;
    std::string err;
    struct Offsets {
        size_t type, uv, nb, k, x[2], y[2], sp[2], id[2], counts, bsum, boff, total, sc;
    } off{};
    size_t ws_need = 0;
    char *ws = nullptr;
    hipStream_t stream = nullptr, cap_stream = nullptr;
    bool fields_set = false, filled = false;
    int par = 0;             // arrays holding the current particles
    long long buf_count = 0;
    long measured = 0;
    int xf = 0;
    long compact_every = 1;
    std::map<std::tuple<long, int, int>, hipGraphExec_t> graphs;
    void *ptr(size_t o) const { return ws + o; }
};

namespace {

using Rw = lbf_rw_s;

lbf_status fail(Rw *r, lbf_status s, const std::string &m)
{
    if (r) r->err = m;
    return s;
}

lbf_status hip_fail(Rw *r, hipError_t e, const char *what)
{
    return fail(r, LBF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

void layout(Rw *r)
{
    const size_t n = (size_t)r->p.nx * r->p.ny, C = (size_t)r->p.capacity;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    r->off.type = take(n);
    r->off.uv = take(16 * n);
    r->off.nb = take(8 * ((size_t)r->p.nx + 6) * ((size_t)r->p.ny + 6));
    r->off.k = take(8 * n);
    for (int b = 0; b < 2; ++b) {
        r->off.x[b] = take(8 * C);
        r->off.y[b] = take(8 * C);
        r->off.sp[b] = take(C);
        r->off.id[b] = take(8 * C);
    }
    r->off.counts = take(4 * n);
    r->off.bsum = take(8 * SCAN_BLOCKS);
    r->off.boff = take(8 * SCAN_BLOCKS);
    r->off.total = take(8);
    r->off.sc = take(sizeof(Scalars));
    r->ws_need = off;
}

Field field(Rw *r)
{
    Field f{};
    f.nx = r->p.nx;
    f.ny = r->p.ny;
    f.ns = r->p.nspecies;
    f.wall_mode = r->p.wall_mode;
    f.type = (const uint8_t *)r->ptr(r->off.type);
    f.uv = (const double2 *)r->ptr(r->off.uv);
    f.nb = (const uint64_t *)r->ptr(r->off.nb);
    f.k = (const double *)r->ptr(r->off.k);
    f.vs = r->p.vel_scale;
    f.dt = r->p.dt;
    f.len = std::sqrt(4.0 * r->p.D * r->p.dt);
    f.zone = r->p.zone;
    f.rate_w = r->p.rate_w;
    f.seed = r->p.seed;
    return f;
}

Parts parts(Rw *r, int b)
{
    return Parts{(double *)r->ptr(r->off.x[b]), (double *)r->ptr(r->off.y[b]),
                 (uint8_t *)r->ptr(r->off.sp[b]), (uint64_t *)r->ptr(r->off.id[b])};
}

// One step from the arrays of parity `par`.  With `compact` the survivors are
// first compacted into the other arrays (order preserved) and the step works
// there; without, it appends to and moves the arrays it found.  Particles do
// not interact, so where the compactions fall changes no result.
hipError_t enqueue_step(Rw *r, int par, int measure, bool compact, hipStream_t s)
{
    Scalars *sc = (Scalars *)r->ptr(r->off.sc);
    long long *bsum = (long long *)r->ptr(r->off.bsum), *boff = (long long *)r->ptr(r->off.boff);
    const Parts src = parts(r, par), dst = parts(r, compact ? par ^ 1 : par);
    const long long C = r->p.capacity;
    if (compact) {
        hipLaunchKernelGGL(k_count_alive, dim3(SCAN_BLOCKS), dim3(SCAN_THREADS), 0, s, src, sc, r->p.nx, bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCKS), 0, s, bsum, boff, &sc->n_alive);
        hipLaunchKernelGGL(k_compact, dim3(SCAN_BLOCKS), dim3(SCAN_THREADS), 0, s, src, dst, sc, r->p.nx, boff);
    }
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(1), 0, s, sc, r->buf_count, C, compact ? 0 : 1);
    hipLaunchKernelGGL(k_insert, dim3(64), dim3(256), 0, s, dst, sc, r->buf_count, C, r->p.seed,
                       0.5, r->p.ny - 1.5);
    const long long gmax = (C + 255) / 256;
    const unsigned grid = (unsigned)(gmax < 8192 ? (gmax > 0 ? gmax : 1) : 8192);
    hipLaunchKernelGGL(k_move, dim3(grid), dim3(256), 0, s, field(r), dst, sc, r->xf + 0.5, measure);
    return hipGetLastError();
}

lbf_status run_block(Rw *r, long n, int measure)
{
    if (n <= 0) return LBF_OK;
    const auto key = std::make_tuple(n, r->par, measure);
    auto it = r->graphs.find(key);
    if (it == r->graphs.end()) {
        hipError_t e = hipStreamBeginCapture(r->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(r, e, "hipStreamBeginCapture");
        int p = r->par;
        hipError_t le = hipSuccess;
        for (long i = 0; i < n && le == hipSuccess; ++i) {
            const bool compact = i % r->compact_every == 0;
            le = enqueue_step(r, p, measure, compact, r->cap_stream);
            if (compact) p ^= 1;
        }
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(r->cap_stream, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(r, le, "step launch during capture");
        }
        if (e != hipSuccess) return hip_fail(r, e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(r, e, "hipGraphInstantiate");
        it = r->graphs.emplace(key, ex).first;
    }
    hipError_t e = hipGraphLaunch(it->second, r->stream);
    if (e != hipSuccess) return hip_fail(r, e, "hipGraphLaunch");
    if (((n + r->compact_every - 1) / r->compact_every) & 1) r->par ^= 1;  // one swap per compaction
    return LBF_OK;
}

lbf_status run_steps(Rw *r, long n, int measure)
{
    while (n > 0) {
        const long m = std::min<long>(n, 200);
        lbf_status st = run_block(r, m, measure);
        if (st != LBF_OK) return st;
        n -= m;
        if (measure) r->measured += m;
    }
    return LBF_OK;
}

lbf_status ready(Rw *r)
{
    if (!r) return LBF_EINVAL;
    if (!r->valid) return fail(r, LBF_EINVAL, "created with invalid parameters");
    if (!r->ws) return fail(r, LBF_ESTATE, "no workspace bound");
    return LBF_OK;
}

}  // namespace

extern "C" {

lbf_status lbf_rw_params_default(lbf_rw_params *p, int nx, int ny)
{
    if (!p) return LBF_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->nx = nx;
    p->ny = ny;
    p->nspecies = 2;
    p->xf = -1;
    p->wall_mode = 1;
    p->D = 0.05;
    p->dt = 0.5;
    p->zone = 1.0;
    p->rate_w = 1.0 / 6.0;
    p->density = 10.0;
    p->vel_scale = 1.0;
    p->seed = 1;
    p->capacity = (long)(p->density * 1.5 * nx * ny) + 4096;
    return LBF_OK;
}

lbf_status lbf_rw_create(const lbf_rw_params *p, lbf_rw *out)
{
    if (!out) return LBF_EINVAL;
    *out = nullptr;
    Rw *r = new (std::nothrow) Rw();
    if (!r) return LBF_ENOMEM;
    *out = r;
    if (!p) return fail(r, LBF_EINVAL, "params is NULL");
    std::string why;
    if (p->nx < 8 || p->ny < 3) why = "need nx >= 8 and ny >= 3";
    else if (p->nspecies != 2 && p->nspecies != 3) why = "nspecies must be 2 or 3";
    else if (p->wall_mode != 0 && p->wall_mode != 1) why = "wall_mode must be 0 or 1";
    else if (!(p->dt > 0) || !(p->D >= 0) || !(std::sqrt(4.0 * p->D * p->dt) < 0.9))
        why = "need dt > 0, D >= 0 and sqrt(4 D dt) < 0.9";
    else if (!(p->zone > 0 && p->zone <= 1)) why = "zone must lie in (0, 1]";
    else if (!(p->density > 0 && p->density <= 200)) why = "density must lie in (0, 200]";
    else if (!(p->vel_scale >= 0) || !(p->rate_w >= 0)) why = "vel_scale and rate_w must be >= 0";
    else if (p->xf != -1 && (p->xf < 0 || p->xf > p->nx - 2)) why = "xf must be -1 or in [0, nx-2]";
    else if (p->capacity < 1 || p->capacity > (1L << 34)) why = "capacity out of range";
    if (!why.empty()) return fail(r, LBF_EINVAL, why);
    r->p = *p;
    r->xf = p->xf == -1 ? p->nx - 3 : p->xf;
    r->compact_every = std::min<long>(COMPACT_MAX, std::max<long>(1, p->nx / 8));
    r->buf_count = std::lround(p->density * (BUF_HI - BUF_LO) * ((p->ny - 1.5) - 0.5));
    layout(r);
    r->valid = true;
    return LBF_OK;
}

lbf_status lbf_rw_workspace_bytes(lbf_rw r, size_t *bytes)
{
    if (!r || !bytes) return LBF_EINVAL;
    if (!r->valid) return fail(r, LBF_EINVAL, "created with invalid parameters");
    *bytes = r->ws_need;
    return LBF_OK;
}

lbf_status lbf_rw_bind(lbf_rw r, void *ws, size_t bytes, void *stream)
{
    if (!r) return LBF_EINVAL;
    if (!r->valid) return fail(r, LBF_EINVAL, "created with invalid parameters");
    if (!ws || (uintptr_t)ws % 256) return fail(r, LBF_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < r->ws_need) return fail(r, LBF_ENOMEM, "workspace smaller than lbf_rw_workspace_bytes");
    for (auto &kv : r->graphs) (void)hipGraphExecDestroy(kv.second);
    r->graphs.clear();
    if (!r->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&r->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(r, e, "hipStreamCreate");
    }
    r->ws = (char *)ws;
    r->stream = (hipStream_t)stream;
    r->fields_set = r->filled = false;
    return LBF_OK;
}

lbf_status lbf_rw_set_fields(lbf_rw r, const uint8_t *type, const double *ux, const double *uy,
                             const double *k)
{
    lbf_status st = ready(r);
    if (st != LBF_OK) return st;
    if (!type || !ux || !uy || !k) return fail(r, LBF_EINVAL, "NULL field");
    const size_t n = (size_t)r->p.nx * r->p.ny;
    std::vector<uint8_t> t(n);
    hipError_t e = hipMemcpyAsync(t.data(), type, n, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(r, e, "copy node_type");
    for (int x = 0; x < r->p.nx; ++x)
        if (t[x] == 0 || t[n - r->p.nx + x] == 0) return fail(r, LBF_EINVAL, "rows 0 and ny-1 must be solid");
    for (uint8_t v : t)
        if (v > 3) return fail(r, LBF_EINVAL, "node_type values must be 0..3");
    const void *src[2] = {type, k};
    const size_t off[2] = {r->off.type, r->off.k};
    const size_t bytes[2] = {n, 8 * n};
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = hipMemcpyAsync(r->ptr(off[i]), src[i], bytes[i], hipMemcpyDeviceToDevice, r->stream);
    if (e != hipSuccess) return hip_fail(r, e, "copy fields");
    const size_t nw = ((size_t)r->p.nx + 6) * ((size_t)r->p.ny + 6);
    const unsigned blocks = (unsigned)std::min<size_t>((nw + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pack_fields, dim3(blocks), dim3(256), 0, r->stream, field(r), ux, uy,
                       (double2 *)r->ptr(r->off.uv), (uint64_t *)r->ptr(r->off.nb));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(r, e, "pack fields");
    r->fields_set = true;
    r->filled = false;
    return LBF_OK;
}

lbf_status lbf_rw_fill(lbf_rw r)
{
    lbf_status st = ready(r);
    if (st != LBF_OK) return st;
    if (!r->fields_set) return fail(r, LBF_ESTATE, "fields not set");
    Scalars *sc = (Scalars *)r->ptr(r->off.sc);
    hipError_t e = hipMemsetAsync(sc, 0, sizeof(Scalars), r->stream);
    int *counts = (int *)r->ptr(r->off.counts);
    long long *bsum = (long long *)r->ptr(r->off.bsum), *boff = (long long *)r->ptr(r->off.boff);
    long long *total = (long long *)r->ptr(r->off.total);
    const long long ncell = (long long)r->p.nx * r->p.ny;
    const Field f = field(r);
    r->par = 0;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fill_count, dim3(1024), dim3(256), 0, r->stream, f, r->p.density, counts);
        hipLaunchKernelGGL(k_fill_sum, dim3(SCAN_BLOCKS), dim3(SCAN_THREADS), 0, r->stream, counts, ncell, bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_BLOCKS), 0, r->stream, bsum, boff, total);
        hipLaunchKernelGGL(k_fill_place, dim3(SCAN_BLOCKS), dim3(SCAN_THREADS), 0, r->stream, f, counts,
                           boff, parts(r, 0), (long long)r->p.capacity, sc);
        hipLaunchKernelGGL(k_fill_finish, dim3(1), dim3(1), 0, r->stream, sc, total,
                           (long long)r->p.capacity);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(r, e, "fill kernels");
    r->filled = true;
    r->measured = 0;
    return LBF_OK;
}

lbf_status lbf_rw_run(lbf_rw r, long nsteps, int measure)
{
    lbf_status st = ready(r);
    if (st != LBF_OK) return st;
    if (!r->filled) return fail(r, LBF_ESTATE, "call lbf_rw_fill first");
    if (nsteps < 0) return fail(r, LBF_EINVAL, "nsteps < 0");
    return run_steps(r, nsteps, measure ? 1 : 0);
}

lbf_status lbf_rw_counts(lbf_rw r, double *N, long *np, long *steps)
{
    lbf_status st = ready(r);
    if (st != LBF_OK) return st;
    if (!r->filled) return fail(r, LBF_ESTATE, "call lbf_rw_fill first");
    Scalars h;
    hipError_t e = hipMemcpyAsync(&h, r->ptr(r->off.sc), sizeof h, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(r, e, "read counters");
    if (h.overflow) return fail(r, LBF_ENOMEM, "particle capacity exceeded");
    if (N)
        for (int s = 0; s < r->p.nspecies; ++s)
            N[s] = r->measured ? (double)h.cross[s] / (r->measured * r->p.dt) : 0.0;
    if (np) *np = (long)h.n_held;
    if (steps) *steps = r->measured;
    return LBF_OK;
}

lbf_status lbf_rw_walk(lbf_rw r, long np, const uint64_t *ids, double *x, double *y, uint8_t *sp,
                       long t0, long steps)
{
    lbf_status st = ready(r);
    if (st != LBF_OK) return st;
    if (!r->fields_set) return fail(r, LBF_ESTATE, "fields not set");
    if (np < 0 || t0 < 0 || steps < 0) return fail(r, LBF_EINVAL, "negative size");
    if (np == 0 || steps == 0) return LBF_OK;
    if (!ids || !x || !y || !sp) return fail(r, LBF_EINVAL, "NULL particle array");
    const long blocks = std::min<long>((np + 255) / 256, 8192);
    hipLaunchKernelGGL(k_walk, dim3((unsigned)blocks), dim3(256), 0, r->stream, field(r), (long long)np,
                       ids, x, y, sp, (long long)t0, (long long)steps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(r, e, "walk kernel");
    return LBF_OK;
}

lbf_status lbf_rw_time_steps(lbf_rw r, long nsteps, int measure, double *ms)
{
    lbf_status st = ready(r);
    if (st != LBF_OK) return st;
    if (!r->filled) return fail(r, LBF_ESTATE, "call lbf_rw_fill first");
    if (nsteps < 1 || !ms) return fail(r, LBF_EINVAL, "need nsteps >= 1 and ms");
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return hip_fail(r, e, "hipEventCreate");
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(r, e, "hipEventCreate");
    }
    e = hipEventRecord(a, r->stream);
    if (e == hipSuccess) st = run_steps(r, nsteps, measure ? 1 : 0);
    if (e == hipSuccess && st == LBF_OK) e = hipEventRecord(b, r->stream);
    if (e == hipSuccess && st == LBF_OK) e = hipEventSynchronize(b);
    float f = 0;
    if (e == hipSuccess && st == LBF_OK) e = hipEventElapsedTime(&f, a, b);
    *ms = f;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != LBF_OK) return st;
    if (e != hipSuccess) return hip_fail(r, e, "timing events");
    return LBF_OK;
}

const char *lbf_rw_last_error(lbf_rw r) { return r ? r->err.c_str() : "NULL handle"; }

void lbf_rw_destroy(lbf_rw r)
{
    if (!r) return;
    for (auto &kv : r->graphs) (void)hipGraphExecDestroy(kv.second);
    if (r->cap_stream) (void)hipStreamDestroy(r->cap_stream);
    delete r;
}

}  // extern "C"
