// Device helpers shared by the stencil kernels: block -> tile mapping.
#pragma once

#include "lbf_internal.hpp"

#include <type_traits>

namespace lbf {

// Map the hardware block to a tile.  Blocks of one launch are handed to the
// 8 XCDs round-robin (block h runs on XCD h mod 8); with xcd_remap the
// blocks of XCD j are given one contiguous range of tiles, so tiles that
// share halo cache lines mostly run under the same L2.
__device__ __forceinline__ void tile_of_index(const Launch &L, int h, int &bx, int &by)
{
    const int nb = L.gx * L.gy;
    int logical = h;
    if (L.xcd_remap) {
        const int q = nb >> 3, r = nb & 7, j = h & 7, k = h >> 3;
        logical = j * q + (j < r ? j : r) + k;
    }
    bx = logical % L.gx;
    by = logical / L.gx;
}

__device__ __forceinline__ void tile_of_block(const Launch &L, int &bx, int &by)
{
    tile_of_index(L, (int)blockIdx.x, bx, by);
}

__device__ __forceinline__ void tile_coords(const Launch &L, int &x, int &y)
{
    int bx, by;
    tile_of_block(L, bx, by);
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

// Reads and writes of a block of population planes at byte offsets from its
// base.  Narrow blocks (< 4 GiB) go through a buffer descriptor (base and
// byte range, wavefront-uniform, in scalar registers) with a 32-bit offset
// per lane: a choice between two sources (bounce-back or neighbour) is then a
// choice of offset and no lane does 64-bit address arithmetic; an offset
// beyond the range reads 0 and drops a store instead of touching memory.
// Word 3 0x00020000 is the raw 32-bit format of a GFX9 descriptor; cache-
// policy bit 1 is the non-temporal hint.  WIDE blocks use a plain pointer
// and 64-bit offsets.
using rsrc_t = __amdgpu_buffer_rsrc_t;

template <bool WIDE>
using off_t_ = typename std::conditional<WIDE, size_t, uint32_t>::type;

template <typename Real, bool NT, bool WIDE>
struct PopBlock;

template <typename Real, bool NT>
struct PopBlock<Real, NT, false> {
    using real_type = Real;
    rsrc_t r;
    __device__ __forceinline__ PopBlock(const Real *base, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<Real *>(base), 0, (int)bytes, 0x00020000))
    {
    }
    __device__ __forceinline__ Real load(uint32_t off) const
    {
        constexpr int aux = NT ? 2 : 0;
        if constexpr (sizeof(Real) == 4)
            return __builtin_bit_cast(Real, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, aux));
        else
            return __builtin_bit_cast(Real, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, aux));
    }
    __device__ __forceinline__ void store(uint32_t off, Real v) const
    {
        constexpr int aux = NT ? 2 : 0;
        if constexpr (sizeof(Real) == 4)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, aux);
        else
            __builtin_amdgcn_raw_buffer_store_b64(
                __builtin_bit_cast(unsigned int __attribute__((ext_vector_type(2))), v), r, off, 0,
                aux);
    }
};

template <typename Real, bool NT>
struct PopBlock<Real, NT, true> {
    using real_type = Real;
    const char *p;
    __device__ __forceinline__ PopBlock(const Real *base, size_t)
        : p(reinterpret_cast<const char *>(base))
    {
    }
    __device__ __forceinline__ Real load(size_t off) const
    {
        return ld<NT>(reinterpret_cast<const Real *>(p + off));
    }
    __device__ __forceinline__ void store(size_t off, Real v) const
    {
        st<NT>(reinterpret_cast<Real *>(const_cast<char *>(p) + off), v);
    }
};

// Populations of a tile held in LDS, addressed like a PopBlock.
template <typename Real>
struct LdsBlock {
    using real_type = Real;
    const Real *base;
    __device__ __forceinline__ Real load(uint32_t off) const
    {
        return *reinterpret_cast<const Real *>(reinterpret_cast<const char *>(base) + off);
    }
};

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
