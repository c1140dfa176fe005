// Device helpers shared by the adjoint's sweep kernels: lane shifts, row
// access through buffer resources, the FP64 wave reductions.
#pragma once

#include "ctqw_internal.hpp"

namespace ctqw {
namespace adj {

__device__ __forceinline__ int wrapi(int x, int n) { int r = x % n; return r < 0 ? r + n : r; }

// Lane l receives lane l + 1's value (lane 63: 0) / lane l - 1's (lane 0: 0).
__device__ __forceinline__ float from_right(float x) { return __builtin_amdgcn_update_dpp(0.0f, x, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ double from_right(double x) { return __builtin_amdgcn_update_dpp(0.0, x, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ float from_left(float x) { return __builtin_amdgcn_update_dpp(0.0f, x, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ double from_left(double x) { return __builtin_amdgcn_update_dpp(0.0, x, 0x138, 0xF, 0xF, true); }

// Im(conj(u) v) in FP64.
template <typename T>
__device__ __forceinline__ double im_uv(T ur, T ui, T vr, T vi) {
    return (double)ur * (double)vi - (double)ui * (double)vr;
}

// Im(conj(u) v) in the state's precision.
template <typename T>
__device__ __forceinline__ T im_t(T ur, T ui, T vr, T vi) {
    return fma(ur, vi, -(ui * vr));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Eight values summed over the wave at once: each exchange step hands the
// partner the half of the values this lane does not keep (xor 32: four,
// xor 16: two, xor 8: one), then three steps sum the one value left.  Lane
// l ends with the total of value (l >> 3) (bits 5, 4, 3 of l pick it), in
// a fixed order of additions.  Ten shuffles instead of 48.
__device__ __forceinline__ double reduce8(const double (&v)[8], int lane) {
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0, b3 = (lane & 8) != 0;
    double w[4], x[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double send = b5 ? v[k] : v[k + 4];
        const double keep = b5 ? v[k + 4] : v[k];
        w[k] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double send = b4 ? w[k] : w[k + 2];
        const double keep = b4 ? w[k + 2] : w[k];
        x[k] = keep + __shfl_xor(send, 16, 64);
    }
    double y = (b3 ? x[1] : x[0]) + __shfl_xor(b3 ? x[0] : x[1], 8, 64);
    y += __shfl_xor(y, 4, 64);
    y += __shfl_xor(y, 2, 64);
    y += __shfl_xor(y, 1, 64);
    return y;
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRawBufferWord3 = 0x00020000;   // gfx9-family raw buffer, no format conversion
constexpr uint32_t kPastEnd = 0x80000000u;    // an offset past every row: loads read 0, stores drop

// One amplitude per lane through a buffer resource over a row.  Stores take
// a zero scalar offset (a 16-byte store reads its data registers after it
// issues; the compiler keeps the wait before the next write of them only
// when the scalar offset is not a register).
__device__ __forceinline__ float2 load_c(__amdgpu_buffer_rsrc_t rs, uint32_t off, float2*) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
__device__ __forceinline__ double2 load_c(__amdgpu_buffer_rsrc_t rs, uint32_t off, double2*) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    return make_double2(__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z));
}
__device__ __forceinline__ void store_c(float re, float im, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x2 v;
    v.x = __float_as_uint(re);
    v.y = __float_as_uint(im);
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, (int)off, 0, 0);
}
__device__ __forceinline__ void store_c(double re, double im, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x4 v;
    v.x = (unsigned)__double2loint(re);
    v.y = (unsigned)__double2hiint(re);
    v.z = (unsigned)__double2loint(im);
    v.w = (unsigned)__double2hiint(im);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, 0);
}

}  // namespace adj
}  // namespace ctqw
