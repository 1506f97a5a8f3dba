// lbf_efficiency_noalloc: the outlet fluxes, the inflow of A and eps of an
// ADR state blob (the layout lbf_get_state writes) without a context, a
// workspace or any device allocation.  Its scratch -- the per-block partial
// sums of the flux reduction and the four final sums staged for the copy to
// the host -- lives in the file-scope device array `scratch`; the host side
// reaches that array only through the address hipGetSymbolAddress returns
// for the current device (one copy per GPU, kept until the process ends).
//
// Paper: Sec. "Boundary conditions and flux computation in ADE" (outflux
// through the plane two nodes before the outlet), Eq. A-B (eps).
#include <cstring>
#include <mutex>

#include "ctx.hpp"

namespace lbf {
namespace {

// Rows per block of the partial flux sums, and the number of blocks the
// scratch holds: lattices of up to NOALLOC_MAX_ROWS rows.
constexpr int NA_ROWS = 64;
constexpr int NA_MAX_BLOCKS = 4096;
constexpr long NOALLOC_MAX_ROWS = (long)NA_ROWS * NA_MAX_BLOCKS;
constexpr int NA_DEVICES = 64;

// [NA_MAX_BLOCKS][4] partial sums (N_A, N_B, N_C, inflow of A), then the 4
// final sums.  128 KiB + 32 B per GPU.
static __device__ __align__(256) double scratch[4 * NA_MAX_BLOCKS + 4];

std::mutex na_mutex;
double *na_ptr[NA_DEVICES] = {};

// Partial sums of block b over rows [b NA_ROWS, (b + 1) NA_ROWS): the net
// population flux of each species through the face between xf and xf + 1
// (rows where both nodes are fluid) and the inflow of A through the inlet
// face, from the post-collision lattice of the last step.  node_type is the
// caller's unpadded [ny][nx] map (0 = fluid).
template <typename Real>
__global__ __launch_bounds__(NA_ROWS) void k_flux_rows(const Real *prev, const uint8_t *type,
                                                       int ns, int nx, int ny, int nxp, size_t P,
                                                       int xf, double cin, double cref,
                                                       double *partial)
{
    __shared__ double sm[4][NA_ROWS];
    const int y = blockIdx.x * NA_ROWS + threadIdx.x;
    double acc[4] = {0, 0, 0, 0};
    if (y < ny) {
        const size_t t = (size_t)y * nx, a = (size_t)y * nxp + xf;
        if (type[t + xf] == 0 && type[t + xf + 1] == 0)
            for (int s = 0; s < ns; ++s)
                acc[s] = (double)prev[(s * 5 + 1) * P + a] - (double)prev[(s * 5 + 3) * P + a + 1];
        if (type[t] == 0)
            acc[3] = 2.0 * (1.0 / 6.0) * (cin - cref) - 2.0 * (double)prev[3 * P + (size_t)y * nxp];
    }
    for (int s = 0; s < 4; ++s) sm[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int st = NA_ROWS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int s = 0; s < 4; ++s) sm[s][threadIdx.x] += sm[s][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 4) partial[4 * blockIdx.x + threadIdx.x] = sm[threadIdx.x][0];
}

// The four totals, summed over the blocks in order (deterministic).
__global__ __launch_bounds__(64) void k_sum_rows(const double *partial, int nblocks, double *out)
{
    if (threadIdx.x >= 4) return;
    double acc = 0;
    for (int b = 0; b < nblocks; ++b) acc += partial[4 * b + threadIdx.x];
    out[threadIdx.x] = acc;
}

// Device address of this GPU's scratch array, looked up once per device
// with that device current.
hipError_t scratch_ptr(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NA_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        na_ptr[dev] = (double *)p;
    }
    *out = na_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace lbf

using namespace lbf;

extern "C" lbf_status lbf_efficiency_noalloc(const lbf_params *p, const void *state_dev,
                                             const uint8_t *node_type_dev, void *hip_stream,
                                             double *eps, double *N, double *inflow_A)
{
    std::string why;
    lbf_status st = validate_params(p, why);
    if (st != LBF_OK) return st;
    if (p->boundary != 0) return LBF_EINVAL;  // a periodic box has no outlet flux
    if (!state_dev || !node_type_dev) return LBF_EINVAL;
    if ((long)p->ny > NOALLOC_MAX_ROWS) return LBF_ENOMEM;  // beyond the scratch
    const int nx = p->nx, ny = p->ny, ns = p->nspecies, R = p->real_bytes;
    const int nxp = (int)align_up((size_t)nx, ROW_ALIGN);
    const size_t P = (size_t)ny * nxp;
    const size_t L = (size_t)ns * 5 * P * R;  // one lattice of the blob
    const int xf = p->flux_col == -1 ? nx - 3 : p->flux_col;
    const double cref = storage_shift(*p);
    hipStream_t s = (hipStream_t)hip_stream;

    // the blob's header must describe a stepped state of this lattice
    int64_t hdr[4];
    hipError_t e = hipMemcpyAsync(hdr, (const char *)state_dev + 2 * L, sizeof hdr,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return LBF_EHIP;
    if (hdr[1] != ns || hdr[2] != R || hdr[3] != (int64_t)P) return LBF_EINVAL;
    if (hdr[0] < 1) return LBF_ESTATE;

    double *sc = nullptr;
    e = scratch_ptr(&sc);
    if (e != hipSuccess) return LBF_EHIP;
    double *partial = sc, *out = sc + 4 * NA_MAX_BLOCKS;
    // the fluxes read the lattice one step back: the blob's second lattice
    const void *prev = (const char *)state_dev + L;
    const int nblk = (ny + NA_ROWS - 1) / NA_ROWS;
    if (R == 4)
        hipLaunchKernelGGL(k_flux_rows<float>, dim3(nblk), dim3(NA_ROWS), 0, s,
                           (const float *)prev, node_type_dev, ns, nx, ny, nxp, P, xf, p->c_in,
                           cref, partial);
    else
        hipLaunchKernelGGL(k_flux_rows<double>, dim3(nblk), dim3(NA_ROWS), 0, s,
                           (const double *)prev, node_type_dev, ns, nx, ny, nxp, P, xf, p->c_in,
                           cref, partial);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(64), 0, s, partial, nblk, out);
    e = hipGetLastError();
    double h[4];
    if (e == hipSuccess) e = hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return LBF_EHIP;
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(h[k])) return LBF_EDIVERGED;
    if (N)
        for (int k = 0; k < ns; ++k) N[k] = h[k];
    if (inflow_A) *inflow_A = h[3];
    if (eps) *eps = efficiency_of(h, ns);
    return LBF_OK;
}
