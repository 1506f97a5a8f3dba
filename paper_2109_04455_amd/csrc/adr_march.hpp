// Two ADR steps per launch by wavefronts that march along y.
//
// A wavefront owns a strip of 64 columns x MARCH_H output rows (one node per
// lane, lanes along x).  It walks the strip's rows one at a time and applies
// step 1 (from the lattice in HBM) to rows y0 - 1 ... y0 + H, keeping the
// step-1 results of the last three rows in registers (rounded to Real exactly
// as a store would round them), and step 2 to the middle row of that window
// as soon as the row after it is done, writing the result to HBM.  Neighbours
// along x come from the adjacent lanes (wavefront-wide DPP shifts); the two
// columns just outside the strip (x0 - 1, x0 + 64) are updated once per strip
// by a ring pass whose lanes each take one (row, side) pair and keep the one
// population that streams into the strip.  The loads of the next row are
// issued before the current row is computed, so every wavefront keeps a row
// of reads in flight while it computes and writes; no LDS tile and no block
// barrier is involved.  Strips alternate their marching direction (up, down)
// so that the halo row two vertically adjacent strips both read is read by
// both near the same time (at the start or at the end of the launch).
//
// Node arithmetic is the code of the single-step kernel (pull, collide,
// react); only where the gathered values come from differs, so the results
// equal those of two single steps.  Link reactions in a channel, FP32
// storage with FP64 node arithmetic, lattices addressed with 32-bit offsets.
// An alternative to the LDS tile of pair_update, selected by flags bit 9:
// with the FP64 node arithmetic a wavefront needs ~150 VGPRs, so three
// wavefronts per SIMD share the VALU, and the dependent FP64 chains of one
// row leave them waiting to issue about half of their cycles (measured on a
// 4096 x 1024 lattice: 155 us per launch against 127 us for the LDS tile).
#pragma once

#include "adr_device.hpp"

namespace lbf {
namespace adr {

constexpr int MARCH_WAVES = 4;   // strips (wavefronts) per block, adjacent in x

// Lane i takes lane i - 1's value, lane 0 takes `edge` (wave_shr:1) / lane i
// takes lane i + 1's value, lane 63 takes `edge` (wave_shl:1).  The edge
// value is the DPP's "old" operand, so no select follows the shift: a shift
// placed in a branch that disables lane 0 (or 63) would read 0 from it.
// Call with every lane active.
__device__ __forceinline__ float from_left(float v, float edge)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138,
                                                      0xF, 0xF, false));
}
__device__ __forceinline__ float from_right(float v, float edge)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130,
                                                      0xF, 0xF, false));
}
__device__ __forceinline__ float lane_f(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double lane_d(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// What step 1 of one node reads from HBM: its mask, velocity and the five
// pulled populations of every species (the bounce-back, inlet and outlet
// choices are choices of offset; at the outlet the W slot holds the node's
// own E population).
template <int S>
struct RowIn {
    unsigned m;
    float u, v;
    float g[S][5];
};

// Byte offset past every buffer range of the lattice: a buffer load there
// returns 0 and a store is dropped, so lanes with nothing to read or write
// take part in the same (branch-free) memory instructions.
constexpr uint32_t OFF_NONE = 0xFFFFFFF0u;

template <int S>
__device__ __forceinline__ void row_issue(const AdrArgs<float> &a, int x, int y, unsigned m,
                                          RowIn<S> &r)
{
    r.m = m;
    constexpr uint32_t B = 4;
    const bool live = m != MASK5_SOLID;
    const uint32_t PB = (uint32_t)a.plane * B, RB = (uint32_t)a.nxp * B;
    const uint32_t o = (uint32_t)((size_t)(y < 0 ? 0 : y) * a.nxp + x) * B;
    const PopBlock<float, false, false> vel(a.ua, 2 * PB);
    r.u = vel.load(live ? o : OFF_NONE);
    r.v = vel.load(live ? o + PB : OFF_NONE);
    const uint32_t oE = o + DE * PB, oN = o + DN * PB, oW = o + DW * PB, oS = o + DS * PB;
    const uint32_t s0 = live ? o : OFF_NONE;
    const uint32_t sE = !live ? OFF_NONE : (x == 0 || (m & BIT_W)) ? oW : oE - B;
    const uint32_t sN = !live ? OFF_NONE : (m & BIT_S) ? oS : oN - RB;
    const uint32_t sW = !live ? OFF_NONE : (x == a.nx - 1 || (m & BIT_E)) ? oE : oW + B;
    const uint32_t sS = !live ? OFF_NONE : (m & BIT_N) ? oN : oS + RB;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const PopBlock<float, false, false> blk(a.src + (size_t)s * 5 * a.plane, 5 * PB);
        r.g[s][0] = blk.load(s0);
        r.g[s][DE] = blk.load(sE);
        r.g[s][DN] = blk.load(sN);
        r.g[s][DW] = blk.load(sW);
        r.g[s][DS] = blk.load(sS);
    }
}

// Store of one node's post-collision populations at byte offset o
// (OFF_NONE: dropped), branch-free.
template <int S, bool NT>
__device__ __forceinline__ void row_store(const AdrArgs<float> &a, uint32_t o, const double (&h)[S][5])
{
    const uint32_t PB = (uint32_t)a.plane * 4;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const PopBlock<float, NT, false> out(a.dst + (size_t)s * 5 * a.plane, 5 * PB);
#pragma unroll
        for (int i = 0; i < 5; ++i) out.store(o == OFF_NONE ? OFF_NONE : o + i * PB, float(h[s][i]));
    }
}

// Pre-collision populations of one node from its loads (the formulas of
// pull5_at); osum: at the outlet, the sum of the node's five own stored
// populations of each species in pull5_at's order.
template <int S>
__device__ __forceinline__ void row_finish(const RowIn<S> &r, int x, int nx, double inlet_e,
                                           const double (&osum)[S], double (&h)[S][5])
{
#pragma unroll
    for (int s = 0; s < S; ++s) {
        h[s][0] = r.g[s][0];
        h[s][DE] = (x == 0 && s == 0) ? inlet_e - double(r.g[s][DE]) : double(r.g[s][DE]);
        h[s][DN] = r.g[s][DN];
        h[s][DW] = x == nx - 1 ? 2.0 * w5<double>(DW) * osum[s] - double(r.g[s][DW])
                               : double(r.g[s][DW]);
        h[s][DS] = r.g[s][DS];
    }
}

// Step-1 result of one row of the window.
template <int S>
struct Z1 {
    unsigned m;
    float u, v;
    float z[S][5];
};

template <int S, bool NT, int DIR, int H>
__device__ __forceinline__ void march_strip(const AdrArgs<float> &a, int x0, int y0)
{
    static_assert(2 * H <= 64 && H + 2 <= 64, "ring lanes of one wavefront");
    // per wavefront: the ring pass's results, read back by every lane
    __shared__ float s_ring[MARCH_WAVES][S][64];
    __shared__ double s_osum[MARCH_WAVES][S][H + 2];
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    const int x = x0 + lane;
    const int nx = a.nx, ny = a.ny;
    const double inlet_e = 2.0 * w5<double>(DE) * (a.cin - a.cref);
    const bool has_outlet = x0 <= nx - 1 && nx - 1 < x0 + 64;

    // step-1 row k of the march (k = 0 ... H + 1); masks come through a
    // buffer descriptor (a row outside the lattice reads 0 and is taken as
    // solid where the mask is used, after the load has landed)
    auto row_of = [&](int k) { return DIR > 0 ? y0 - 1 + k : y0 + H - k; };
    auto in_lattice = [&](int k) { return k < H + 2 && row_of(k) >= 0 && row_of(k) < ny; };
    const rsrc_t mrs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(a.mask5), 0,
                                                         (int)a.plane, 0x00020000);
    auto mask_load = [&](int k) -> unsigned {
        const uint32_t o = in_lattice(k) ? (uint32_t)((size_t)row_of(k) * a.nxp + x) : OFF_NONE;
        return __builtin_amdgcn_raw_buffer_load_b8(mrs, o, 0, 0);
    };
    auto mask_of = [&](int k, unsigned raw) { return in_lattice(k) ? raw : MASK5_SOLID; };

    // the first two rows' loads go out before the ring pass
    RowIn<S> inA, inB, inC;
    unsigned mA = mask_load(2), mB = 0, mC = 0;
    row_issue<S>(a, x, row_of(0), mask_of(0, mask_load(0)), inA);
    row_issue<S>(a, x, row_of(1), mask_of(1, mask_load(1)), inB);

    // ---- ring pass: the inward population of columns x0 - 1 (even lanes)
    // and x0 + 64 (odd lanes) at output row y0 + lane / 2; in the strip that
    // holds the outlet, lanes 0 ... H + 1 also sum the outlet node's own
    // populations at rows y0 - 1 ... y0 + H
    {
        float ring[S];
#pragma unroll
        for (int s = 0; s < S; ++s) ring[s] = 0.f;
        if (lane < 2 * H) {
            const int yr = y0 + (lane >> 1), xr = (lane & 1) ? x0 + 64 : x0 - 1;
            if (yr < ny && xr >= 0 && xr < nx) {
                const size_t id = (size_t)yr * a.nxp + xr;
                const unsigned m = a.mask5[id];
                if (m != MASK5_SOLID) {
                    double h[S][5];
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        pull5<float, double, false, false>(a.src + (size_t)s * 5 * a.plane, a.plane,
                                                           id, xr, nx, a.nxp, m, s == 0, inlet_e, h[s]);
                    collide_react<float, double, S, false>(a, id, m, double(a.ua[id]),
                                                           double(a.ua[a.plane + id]), h);
#pragma unroll
                    for (int s = 0; s < S; ++s) ring[s] = float(h[s][(lane & 1) ? DW : DE]);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) s_ring[wv][s][lane] = ring[s];
        if (has_outlet && lane < H + 2) {
            const int yo = y0 - 1 + lane;
            double o[S];
#pragma unroll
            for (int s = 0; s < S; ++s) o[s] = 0.0;
            if (yo >= 0 && yo < ny) {
                const size_t id = (size_t)yo * a.nxp + (nx - 1);
                if (a.mask5[id] != MASK5_SOLID)
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        const float *g = a.src + (size_t)s * 5 * a.plane + id;
                        const size_t P = a.plane;
                        o[s] = double(g[0]) + double(g[DE * P]) + double(g[DN * P]) +
                               double(g[DW * P]) + double(g[DS * P]);
                    }
            }
#pragma unroll
            for (int s = 0; s < S; ++s) s_osum[wv][s][lane] = o[s];
        }
    }

    // the window: row k - 1 (zc) and the population row k - 2 passes on to
    // it (its N population when marching up, its S population when down)
    Z1<S> zc;
    float pass[S];
#pragma unroll
    for (int s = 0; s < S; ++s) pass[s] = 0.f;
    zc.m = MASK5_SOLID;

    // one row of the march: load row k + 3's mask into m3, issue row k + 2
    // (mask m2, loaded one row earlier) into `nxt`, step 1 on row k from
    // `cur` (row k + 1 stays in flight), step 2 on row k - 1
    auto body = [&](int k, RowIn<S> &cur, RowIn<S> &nxt, unsigned m2, unsigned &m3) {
        const int yk = row_of(k);
        m3 = mask_load(k + 3);
        if (k + 2 < H + 2) row_issue<S>(a, x, row_of(k + 2), mask_of(k + 2, m2), nxt);

        // step 1 on row k
        Z1<S> zn;
        zn.m = cur.m;
        zn.u = cur.u;
        zn.v = cur.v;
        if (cur.m != MASK5_SOLID) {
            double osum[S];
#pragma unroll
            for (int s = 0; s < S; ++s) osum[s] = has_outlet ? s_osum[wv][s][yk - (y0 - 1)] : 0.0;
            double h[S][5];
            row_finish<S>(cur, x, nx, inlet_e, osum, h);
            const size_t id = (size_t)yk * a.nxp + x;
            collide_react<float, double, S, false>(a, id, cur.m, double(cur.u), double(cur.v), h);
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int i = 0; i < 5; ++i) zn.z[s][i] = float(h[s][i]);
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s)
#pragma unroll
                for (int i = 0; i < 5; ++i) zn.z[s][i] = 0.f;
        }

        // step 2 on row k - 1 (the output rows are k - 1 = 1 ... H)
        if (k >= 2) {
            const int yr = row_of(k - 1);
            const int ri = yr - y0;  // output row index 0 ... H - 1
            // neighbours along x: shifts with every lane active; the strip's
            // edge columns take the ring pass's populations
            float zE[S], zW[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                zE[s] = from_left(zc.z[s][DE], s_ring[wv][s][2 * ri]);
                zW[s] = from_right(zc.z[s][DW], s_ring[wv][s][2 * ri + 1]);
            }
            const unsigned m = zc.m;
            const bool live = m != MASK5_SOLID && yr < ny;
            double h[S][5];
            if (live) {
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    h[s][0] = zc.z[s][0];
                    // E arrives from x - 1
                    if (x == 0)
                        h[s][DE] = s == 0 ? inlet_e - double(zc.z[s][DW]) : double(zc.z[s][DW]);
                    else
                        h[s][DE] = (m & BIT_W) ? double(zc.z[s][DW]) : double(zE[s]);
                    // N arrives from y - 1, S from y + 1
                    const float fromN = DIR > 0 ? pass[s] : zn.z[s][DN];
                    const float fromS = DIR > 0 ? zn.z[s][DS] : pass[s];
                    h[s][DN] = (m & BIT_S) ? double(zc.z[s][DS]) : double(fromN);
                    h[s][DS] = (m & BIT_N) ? double(zc.z[s][DN]) : double(fromS);
                    // W arrives from x + 1
                    if (x == nx - 1) {
                        const double sum = double(zc.z[s][0]) + double(zc.z[s][DE]) +
                                           double(zc.z[s][DN]) + double(zc.z[s][DW]) +
                                           double(zc.z[s][DS]);
                        h[s][DW] = 2.0 * w5<double>(DW) * sum - double(zc.z[s][DE]);
                    } else {
                        h[s][DW] = (m & BIT_E) ? double(zc.z[s][DE]) : double(zW[s]);
                    }
                }
                const size_t id = (size_t)yr * a.nxp + x;
                collide_react<float, double, S, false>(a, id, m, double(zc.u), double(zc.v), h);
            } else {
#pragma unroll
                for (int s = 0; s < S; ++s)
#pragma unroll
                    for (int i = 0; i < 5; ++i) h[s][i] = 0.0;
            }
            row_store<S, NT>(a, live ? (uint32_t)((size_t)yr * a.nxp + x) * 4 : OFF_NONE, h);
        }
        // slide the window: row k - 1 passes on the population streaming
        // into the next middle row
#pragma unroll
        for (int s = 0; s < S; ++s) pass[s] = DIR > 0 ? zc.z[s][DN] : zc.z[s][DS];
        zc = zn;
    };

    // three row buffers in rotation: the loads of the next two rows are in
    // flight while a row is computed; fully unrolled, so no register holding
    // a load in flight is ever copied
    static_assert((H + 2) % 3 == 0, "rows of a strip in whole rotations of three buffers");
#pragma unroll
    for (int k = 0; k < H + 2; k += 3) {
        body(k, inA, inC, mA, mB);
        body(k + 1, inB, inA, mB, mC);
        body(k + 2, inC, inB, mC, mA);
    }
}

}  // namespace adr
}  // namespace lbf
