// Memory-bandwidth probes: what the memory system sustains for a flat copy
// and for the step kernel's access pattern with the arithmetic taken out.
// They put the step kernels' rates beside attainable ones; no part of the
// method runs here.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "../../include/ctqw.h"
#include "ctqw_internal.hpp"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One 16-byte element per thread, stored non-temporal.
__global__ __launch_bounds__(256) void probe_flat_kernel(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                         int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(src[i], dst + i);
}

// One wave per band of 128 complex64 columns (1 KiB of a row) of one n x n
// grid, copying the band row by row with two rows of loads in flight.
// Consecutive waves take the same band of consecutive grids.  The dynamic
// LDS the launch reserves only caps the resident waves per CU.
__global__ __launch_bounds__(64) void probe_band_sweep_kernel(const f32x4* __restrict__ src,
                                                              f32x4* __restrict__ dst, int32_t n, int64_t grids) {
    extern __shared__ char cap[];
    const int64_t g = blockIdx.x % grids;
    const int64_t band = blockIdx.x / grids;
    const int64_t rs = n / 2;                       // row stride in 16-byte elements
    const int64_t off = g * n * rs + band * 64 + threadIdx.x;
    const f32x4* s = src + off;
    f32x4* d = dst + off;
    f32x4 r0 = s[0], r1 = s[rs];
    for (int32_t row = 0; row < n; row += 2) {      // n is even
        const f32x4 v0 = r0, v1 = r1;
        if (row + 2 < n) {
            r0 = s[(int64_t)(row + 2) * rs];
            r1 = s[(int64_t)(row + 3) * rs];
        }
        __builtin_nontemporal_store(v0, d + (int64_t)row * rs);
        __builtin_nontemporal_store(v1, d + (int64_t)(row + 1) * rs);
    }
    if (threadIdx.x >= 64) cap[0] = 0;              // never taken (64-thread blocks)
}

constexpr int kLdsPerCu = 160 * 1024;

}  // namespace

extern "C" ctqw_status ctqw_bandwidth_probe(const void* src, void* dst, int64_t bytes, int32_t pattern, int32_t n,
                                            int32_t waves_per_cu, void* hip_stream) {
    if (!src || !dst || bytes <= 0)
        return (ctqw_status)ctqw::report_error(CTQW_ERR_INVALID_ARG, "ctqw_bandwidth_probe: NULL buffer or bytes <= 0");
    const char* s0 = static_cast<const char*>(src);
    const char* d0 = static_cast<const char*>(dst);
    if (s0 < d0 + bytes && d0 < s0 + bytes)
        return (ctqw_status)ctqw::report_error(CTQW_ERR_INVALID_ARG, "ctqw_bandwidth_probe: src and dst overlap");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const f32x4* a = static_cast<const f32x4*>(src);
    f32x4* b = static_cast<f32x4*>(dst);
    if (pattern == 0) {
        if (bytes % 16 != 0 || (bytes / 16 + 255) / 256 > INT32_MAX)
            return (ctqw_status)ctqw::report_error(CTQW_ERR_INVALID_ARG,
                                                   "ctqw_bandwidth_probe: flat copy needs a multiple of 16 bytes");
        const int64_t elems = bytes / 16;
        hipLaunchKernelGGL(probe_flat_kernel, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, stream, a, b,
                           elems);
    } else if (pattern == 1) {
        if (waves_per_cu == 0) waves_per_cu = 8;
        if (n < 128 || n % 128 != 0 || n > 65536 || waves_per_cu < 4 || waves_per_cu > 32)
            return (ctqw_status)ctqw::report_error(
                CTQW_ERR_INVALID_ARG, "ctqw_bandwidth_probe: band sweep needs n a multiple of 128 and 4..32 waves per CU");
        const int64_t grid_bytes = (int64_t)n * n * 8;
        if (bytes % grid_bytes != 0)
            return (ctqw_status)ctqw::report_error(CTQW_ERR_INVALID_ARG,
                                                   "ctqw_bandwidth_probe: bytes is not a whole number of n x n grids");
        const int64_t grids = bytes / grid_bytes;
        const int64_t waves = grids * (n / 128);
        if (waves >= (int64_t)1 << 31)
            return (ctqw_status)ctqw::report_error(CTQW_ERR_INVALID_ARG, "ctqw_bandwidth_probe: too many bands");
        const size_t lds = waves_per_cu >= 32 ? 0 : (size_t)(kLdsPerCu / waves_per_cu) & ~size_t(255);
        hipLaunchKernelGGL(probe_band_sweep_kernel, dim3((unsigned)waves), dim3(64), lds, stream, a, b, n, grids);
    } else {
        return (ctqw_status)ctqw::report_error(CTQW_ERR_INVALID_ARG, "ctqw_bandwidth_probe: pattern is 0 or 1");
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        char msg[256];
        snprintf(msg, sizeof msg, "ctqw_bandwidth_probe: launch failed: %s", hipGetErrorString(e));
        return (ctqw_status)ctqw::report_error(CTQW_ERR_DEVICE, msg);
    }
    return CTQW_OK;
}
