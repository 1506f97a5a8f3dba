// Device helpers shared by the stencil kernels: block -> tile mapping.
#pragma once

#include "lbf_internal.hpp"

namespace lbf {

// Map the hardware block to a tile.  Blocks of one launch are handed to the
// 8 XCDs round-robin (block h runs on XCD h mod 8); with xcd_remap the
// blocks of XCD j are given one contiguous range of tiles, so tiles that
// share halo cache lines mostly run under the same L2.
__device__ __forceinline__ void tile_coords(const Launch &L, int &x, int &y)
{
    const int nb = L.gx * L.gy;
    const int h = blockIdx.x;
    int logical = h;
    if (L.xcd_remap) {
        const int q = nb >> 3, r = nb & 7, j = h & 7, k = h >> 3;
        logical = j * q + (j < r ? j : r) + k;
    }
    const int bx = logical % L.gx, by = logical / L.gx;
    const int t = threadIdx.x;
    x = bx * L.tx + t % L.tx;
    y = by * L.ty + t / L.tx;
}

// Population loads/stores.  NT selects the non-temporal (streaming) cache
// policy: every population is touched once per step, so there is nothing to
// keep in the caches beyond the halo lines shared inside a wavefront.
template <bool NT, typename Real>
__device__ __forceinline__ Real ld(const Real *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT, typename Real>
__device__ __forceinline__ void st(Real *p, Real v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

inline Launch make_launch(int nx, int ny, int tx, int ty)
{
    Launch L;
    L.tx = tx > 0 ? tx : 64;
    L.ty = ty > 0 ? ty : 4;
    L.gx = (nx + L.tx - 1) / L.tx;
    L.gy = (ny + L.ty - 1) / L.ty;
    return L;
}

}  // namespace lbf
