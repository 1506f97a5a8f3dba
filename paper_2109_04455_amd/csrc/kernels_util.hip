// Set-up kernels (node masks, the list of fluid nodes next to catalysts, the
// rate map) and a plain device copy used as the bandwidth probe.
#include "lbf_internal.hpp"

namespace lbf {
namespace {

constexpr int CX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Per node: padded copy of the node type, the D2Q5 mask (solid and
// catalytic neighbours along E, N, W, S) and the D2Q9 mask (solid
// neighbours along the 8 moving directions).  Neighbours outside the
// channel in y count as solid; outside in x they are the open inlet/outlet.
// A periodic box wraps both directions.
__global__ void k_masks(const uint8_t *type_in, uint8_t *type_pad, uint8_t *mask5, uint16_t *mask9,
                        int nx, int ny, int nxp, int nspecies, bool periodic)
{
    const size_t n = (size_t)nxp * ny;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nxp), y = (int)(i / nxp);
        if (x >= nx) {
            type_pad[i] = 1;
            mask5[i] = MASK5_SOLID;
            mask9[i] = MASK9_SOLID;
            continue;
        }
        const uint8_t t = type_in[(size_t)y * nx + x];
        type_pad[i] = t;
        if (t != 0) {
            mask5[i] = MASK5_SOLID;
            mask9[i] = MASK9_SOLID;
            continue;
        }
        unsigned m9 = 0, m5 = 0;
        for (int d = 1; d < 9; ++d) {
            int sx = x + CX9[d], sy = y + CY9[d];
            if (periodic) {
                sx = (sx + nx) % nx;
                sy = (sy + ny) % ny;
            }
            bool solid, cat = false;
            if (sy < 0 || sy >= ny) {
                solid = true;
            } else if (sx < 0 || sx >= nx) {
                solid = false;
            } else {
                const uint8_t tn = type_in[(size_t)sy * nx + sx];
                solid = tn != 0;
                cat = tn == 2 || (tn == 3 && nspecies == 3);
            }
            if (solid) m9 |= 1u << (d - 1);
            if (d < 5) {
                if (solid) m5 |= 1u << (d - 1);
                if (cat) m5 |= 1u << (d + 3);
            }
        }
        mask5[i] = (uint8_t)m5;
        mask9[i] = (uint16_t)m9;
    }
}

// Fluid nodes with at least one catalytic neighbour get a slot in the trace
// list (order of slots is arbitrary; nothing depends on it).
__global__ void k_trace_list(const uint8_t *mask5, int32_t *trace_idx, int32_t *trace_nodes,
                             int *counter, int nx, int ny, int nxp)
{
    const size_t n = (size_t)nxp * ny;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint8_t m = mask5[i];
        int32_t slot = -1;
        if (m != MASK5_SOLID && (m & 0xF0u)) {
            slot = atomicAdd(counter, 1);
            trace_nodes[slot] = (int32_t)i;
        }
        trace_idx[i] = slot;
    }
}

template <typename Real>
__global__ void k_copy_rates(const double *k_in, const uint8_t *type_pad, Real *kr, int nx, int ny,
                             int nxp)
{
    const size_t n = (size_t)nxp * ny;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nxp), y = (int)(i / nxp);
        const uint8_t t = type_pad[i];
        kr[i] = (x < nx && (t == 2 || t == 3)) ? Real(k_in[(size_t)y * nx + x]) : Real(0);
    }
}

// Streaming copy (the bandwidth probe): 16-byte non-temporal loads and
// stores, four in flight per thread before the first store.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const u32x4 *src, u32x4 *dst, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(src + i);
        const u32x4 b = __builtin_nontemporal_load(src + i + stride);
        const u32x4 c = __builtin_nontemporal_load(src + i + 2 * stride);
        const u32x4 d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void k_copy_bytes(const uint8_t *src, uint8_t *dst, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

hipError_t launch_masks(const uint8_t *type_in, uint8_t *type_pad, uint8_t *mask5, uint16_t *mask9,
                        int nx, int ny, int nxp, int nspecies, bool periodic, hipStream_t s)
{
    hipLaunchKernelGGL(k_masks, dim3(2048), dim3(256), 0, s, type_in, type_pad, mask5, mask9, nx, ny,
                       nxp, nspecies, periodic);
    return hipGetLastError();
}

hipError_t launch_trace_list(const uint8_t *mask5, int32_t *trace_idx, int32_t *trace_nodes,
                             int *counter, int nx, int ny, int nxp, hipStream_t s)
{
    hipLaunchKernelGGL(k_trace_list, dim3(2048), dim3(256), 0, s, mask5, trace_idx, trace_nodes,
                       counter, nx, ny, nxp);
    return hipGetLastError();
}

hipError_t launch_copy_rates(const double *k_in, const uint8_t *type_pad, void *kr, int real_bytes,
                             int nx, int ny, int nxp, hipStream_t s)
{
    if (real_bytes == 4)
        hipLaunchKernelGGL(k_copy_rates<float>, dim3(2048), dim3(256), 0, s, k_in, type_pad,
                           (float *)kr, nx, ny, nxp);
    else
        hipLaunchKernelGGL(k_copy_rates<double>, dim3(2048), dim3(256), 0, s, k_in, type_pad,
                           (double *)kr, nx, ny, nxp);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t nbytes, hipStream_t s)
{
    if (((uintptr_t)src | (uintptr_t)dst | nbytes) % 16 == 0) {
        const size_t n16 = nbytes / 16;
        // 8192 blocks (32 per CU) of 256 threads, each thread four 16-byte
        // transfers per pass
        size_t blocks = (n16 + 1023) / 1024;
        if (blocks > 8192) blocks = 8192;
        if (blocks == 0) blocks = 1;
        hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const u32x4 *)src,
                           (u32x4 *)dst, n16);
    } else {
        hipLaunchKernelGGL(k_copy_bytes, dim3(4096), dim3(256), 0, s, (const uint8_t *)src,
                           (uint8_t *)dst, nbytes);
    }
    return hipGetLastError();
}

}  // namespace lbf
