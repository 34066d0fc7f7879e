// Measured ceilings of the device, for the roofline figures: streaming copy, read and write
// bandwidth of HBM, and the sustained FP64 MFMA and FP64 FMA rates.  These kernels take part
// in no factorization; they are the yardsticks the kernels of a pass are compared with.
#include "scqr_internal.h"

namespace scqr {
namespace {

typedef double d2v __attribute__((ext_vector_type(2)));

// Streaming copy of n16 16-byte chunks: each thread moves U chunks per step (all loads issued
// before the stores), grid-stride over the buffer.  NT: non-temporal stores.
template <int U, bool NT>
__global__ void __launch_bounds__(256) k_peak_copy(const d2v *__restrict__ src, d2v *__restrict__ dst, int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * 256 * U;
    for (int64_t base = (int64_t)blockIdx.x * 256 * U + threadIdx.x; base < n16; base += stride) {
        d2v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + (int64_t)u * 256;
            v[u] = i < n16 ? src[i] : (d2v){0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + (int64_t)u * 256;
            if (i < n16) {
                if (NT)
                    __builtin_nontemporal_store(v[u], dst + i);
                else
                    dst[i] = v[u];
            }
        }
    }
}

// Streaming read: every chunk is loaded and folded into a per-thread sum, written once.
template <int U>
__global__ void __launch_bounds__(256) k_peak_read(const d2v *__restrict__ src, int64_t n16, double *__restrict__ sink)
{
    const int64_t stride = (int64_t)gridDim.x * 256 * U;
    d2v acc = {0.0, 0.0};
    for (int64_t base = (int64_t)blockIdx.x * 256 * U + threadIdx.x; base < n16; base += stride) {
        d2v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + (int64_t)u * 256;
            v[u] = i < n16 ? src[i] : (d2v){0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc.x + acc.y;
}

// Streaming write of a constant.
template <int U, bool NT>
__global__ void __launch_bounds__(256) k_peak_write(d2v *__restrict__ dst, int64_t n16, double val)
{
    const int64_t stride = (int64_t)gridDim.x * 256 * U;
    const d2v v = {val, val};
    for (int64_t base = (int64_t)blockIdx.x * 256 * U + threadIdx.x; base < n16; base += stride) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + (int64_t)u * 256;
            if (i < n16) {
                if (NT)
                    __builtin_nontemporal_store(v, dst + i);
                else
                    dst[i] = v;
            }
        }
    }
}

// FP64 MFMA 16x16x4: ACC independent accumulators per wave, iters rounds of ACC instructions.
template <int ACC>
__global__ void __launch_bounds__(256) k_peak_mfma64(int iters, double seed, double *__restrict__ sink)
{
    d4 acc[ACC];
#pragma unroll
    for (int a = 0; a < ACC; ++a) acc[a] = (d4){0.0, 0.0, 0.0, 0.0};
    const double x = seed * (1.0 + threadIdx.x * 1e-9), y = seed * (1.0 - threadIdx.x * 1e-9);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int a = 0; a < ACC; ++a) acc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[a], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < ACC; ++a) s += acc[a][0] + acc[a][1] + acc[a][2] + acc[a][3];
    sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// FP64 FMA on the vector ALU: CH independent chains per lane.
template <int CH>
__global__ void __launch_bounds__(256) k_peak_fma64(int iters, double seed, double *__restrict__ sink)
{
    double c[CH];
#pragma unroll
    for (int a = 0; a < CH; ++a) c[a] = seed * (a + 1);
    const double m = 1.0 - 1e-12 * (threadIdx.x + 1), d = seed * 1e-3;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int a = 0; a < CH; ++a) c[a] = __builtin_fma(c[a], m, d);
    }
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < CH; ++a) s += c[a];
    sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

template <int U, bool NT>
hipError_t copy_v(hipStream_t s, const void *src, void *dst, int64_t n16, int grid)
{
    hipLaunchKernelGGL((k_peak_copy<U, NT>), dim3(grid), dim3(256), 0, s, static_cast<const d2v *>(src),
                       static_cast<d2v *>(dst), n16);
    return hipGetLastError();
}

template <int U, bool NT>
hipError_t write_v(hipStream_t s, void *dst, int64_t n16, int grid)
{
    hipLaunchKernelGGL((k_peak_write<U, NT>), dim3(grid), dim3(256), 0, s, static_cast<d2v *>(dst), n16, 1.0);
    return hipGetLastError();
}

}  // namespace
}  // namespace scqr

using namespace scqr;

extern "C" {

// variant: bits 0-1 select U = 1, 2, 4, 8 chunks per thread and step; bit 2 non-temporal
// stores.  grid: workgroups of 256 threads (0: 8 per compute unit of a 256-CU device).
scqr_status scqr_peak_copy(void *stream, const void *src, void *dst, int64_t nbytes, int32_t variant, int32_t grid)
{
    if (!src || !dst || nbytes <= 0 || (nbytes & 15) || variant < 0 || variant > 7 || grid < 0) return SCQR_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) return SCQR_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n16 = nbytes / 16;
    const int g = grid ? grid : 2048;
    hipError_t e;
    switch (variant) {
    case 0: e = copy_v<1, false>(s, src, dst, n16, g); break;
    case 1: e = copy_v<2, false>(s, src, dst, n16, g); break;
    case 2: e = copy_v<4, false>(s, src, dst, n16, g); break;
    case 3: e = copy_v<8, false>(s, src, dst, n16, g); break;
    case 4: e = copy_v<1, true>(s, src, dst, n16, g); break;
    case 5: e = copy_v<2, true>(s, src, dst, n16, g); break;
    case 6: e = copy_v<4, true>(s, src, dst, n16, g); break;
    default: e = copy_v<8, true>(s, src, dst, n16, g); break;
    }
    return e == hipSuccess ? SCQR_OK : SCQR_E_HIP;
}

// Streaming read of nbytes; sink receives grid * 256 doubles (grid 0: 2048).
scqr_status scqr_peak_read(void *stream, const void *src, int64_t nbytes, int32_t variant, int32_t grid, double *sink)
{
    if (!src || !sink || nbytes <= 0 || (nbytes & 15) || variant < 0 || variant > 3 || grid < 0) return SCQR_E_INVALID;
    if (reinterpret_cast<uintptr_t>(src) & 15) return SCQR_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n16 = nbytes / 16;
    const int g = grid ? grid : 2048;
    const d2v *p = static_cast<const d2v *>(src);
    switch (variant) {
    case 0: hipLaunchKernelGGL((k_peak_read<1>), dim3(g), dim3(256), 0, s, p, n16, sink); break;
    case 1: hipLaunchKernelGGL((k_peak_read<2>), dim3(g), dim3(256), 0, s, p, n16, sink); break;
    case 2: hipLaunchKernelGGL((k_peak_read<4>), dim3(g), dim3(256), 0, s, p, n16, sink); break;
    default: hipLaunchKernelGGL((k_peak_read<8>), dim3(g), dim3(256), 0, s, p, n16, sink); break;
    }
    return hipGetLastError() == hipSuccess ? SCQR_OK : SCQR_E_HIP;
}

// Streaming write of nbytes (variant as for the copy).
scqr_status scqr_peak_write(void *stream, void *dst, int64_t nbytes, int32_t variant, int32_t grid)
{
    if (!dst || nbytes <= 0 || (nbytes & 15) || variant < 0 || variant > 7 || grid < 0) return SCQR_E_INVALID;
    if (reinterpret_cast<uintptr_t>(dst) & 15) return SCQR_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n16 = nbytes / 16;
    const int g = grid ? grid : 2048;
    hipError_t e;
    switch (variant) {
    case 0: e = write_v<1, false>(s, dst, n16, g); break;
    case 1: e = write_v<2, false>(s, dst, n16, g); break;
    case 2: e = write_v<4, false>(s, dst, n16, g); break;
    case 3: e = write_v<8, false>(s, dst, n16, g); break;
    case 4: e = write_v<1, true>(s, dst, n16, g); break;
    case 5: e = write_v<2, true>(s, dst, n16, g); break;
    case 6: e = write_v<4, true>(s, dst, n16, g); break;
    default: e = write_v<8, true>(s, dst, n16, g); break;
    }
    return e == hipSuccess ? SCQR_OK : SCQR_E_HIP;
}

// FP64 MFMA (16x16x4, 2048 flops per instruction per wave) or FP64 FMA (2 flops per lane per
// instruction) throughput: grid workgroups of 4 waves, each running `iters` rounds of 8
// independent instructions.  sink receives grid * 256 doubles.  kind 0: MFMA, 1: FMA.
scqr_status scqr_peak_fp64(void *stream, int32_t kind, int32_t iters, int32_t grid, double *sink)
{
    if (!sink || iters <= 0 || grid <= 0 || kind < 0 || kind > 1) return SCQR_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (kind == 0)
        hipLaunchKernelGGL((k_peak_mfma64<8>), dim3(grid), dim3(256), 0, s, iters, 1.0 / 3.0, sink);
    else
        hipLaunchKernelGGL((k_peak_fma64<8>), dim3(grid), dim3(256), 0, s, iters, 1.0 / 3.0, sink);
    return hipGetLastError() == hipSuccess ? SCQR_OK : SCQR_E_HIP;
}

}  // extern "C"
