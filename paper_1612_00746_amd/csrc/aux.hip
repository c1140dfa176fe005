// Auxiliary kernels: start state, per-step FP64 norm / truncation check,
// ensemble-averaged observables, rescaling.
#include "ctqw_internal.hpp"

namespace ctqw {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int64_t tri_index(int q, int c, int N) {
    return (int64_t)q * N - ((int64_t)q * (q + 1)) / 2 + c;
}

// p(q, c) = |psi(q, c)|^2 in FP64 for a realisation, any layout.
template <typename C>
__device__ __forceinline__ double prob(const C* __restrict__ psi, const RealDev& rd, int q, int c) {
    const bool tri = (rd.flags & RF_TRIANGLE) != 0;
    int64_t idx;
    if (tri) {
        const int a = q < c ? q : c, b = q < c ? c : q;
        idx = tri_index(a, b, rd.N);
    } else {
        idx = (int64_t)q * rd.N + c;
    }
    const C v = psi[rd.state_off + idx];
    const double re = v.x, im = v.y;
    return re * re + im * im;
}

// ---------------------------------------------------------------- fill / init

__global__ void fill_zero_kernel(uint32_t* __restrict__ p, int64_t words) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = 0u;
}

template <typename C>
__global__ void init_sites_kernel(InitArgs a) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R) return;
    const RealDev rd = a.reals[r];
    const int32_t* s = a.sites + (a.per_real ? r * a.m : 0);
    C* psi = reinterpret_cast<C*>(a.psi) + rd.state_off;
    C one;
    one.x = 1;
    one.y = 0;
    if (a.m == 1) {
        psi[s[0]] = one;
        return;
    }
    if (a.m == 3) {
        psi[((int64_t)s[0] * rd.N + s[1]) * rd.N + s[2]] = one;
        return;
    }
    int x1 = s[0], x2 = s[1];
    if (rd.flags & RF_TRIANGLE) {
        // bosons: phi(x1, x2) = phi(x2, x1) = 1/sqrt 2 (1 on the diagonal);
        // fermions: phi(x1, x2) = -phi(x2, x1) = 1/sqrt 2 for particle 1 on x1
        const bool swapped = x1 > x2;
        if (swapped) { const int t = x1; x1 = x2; x2 = t; }
        C v;
        v.x = (x1 == x2) ? 1.0 : 0.70710678118654752440;
        if ((rd.flags & RF_FERMION) && swapped) v.x = -v.x;
        v.y = 0;
        psi[tri_index(x1, x2, rd.N)] = v;
    } else {
        psi[(int64_t)x1 * rd.N + x2] = one;
    }
}

// ------------------------------------------------------------ step finalize

// One wave per realisation: lane l sums the partials l, l + 64, ... of its
// realisation, then a fixed butterfly combines the lanes (deterministic;
// three walkers have 65536 partials per realisation at N = 256).
__global__ void finalize_kernel(FinalizeArgs a) {
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= a.R) return;   // wave-uniform
    double s = 0.0, t = 0.0;
    for (int32_t k = a.item_first[r] + lane; k < a.item_first[r + 1]; k += 64) {
        s += a.norm_part[k];
        t += a.tail_part[k];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        t += __shfl_xor(t, off, 64);
    }
    if (lane != 0) return;
    const double tf = a.use_max ? a.reals[r].tail_factor_max : a.reals[r].tail_factor;
    const double err2 = t * tf * tf;
    a.norm2[r] = s;
    a.tail2[r] = err2;
    int flag = 0;
    if (a.tol2 > 0.0 && !(err2 <= a.tol2 * s)) flag |= 1;
    if (!isfinite(s) || !isfinite(t)) flag |= 2;
    if (a.norm_alarm > 0.0 && !(fabs(sqrt(s) - 1.0) <= a.norm_alarm)) flag |= 2;
    if (flag) {
        atomicOr(&a.status[0], flag);
        atomicAdd(&a.status[1], 1);
    }
    if (a.renormalize && s > 0.0 && isfinite(s)) a.scale[r] = 1.0 / sqrt(s);
}

// ------------------------------------------------------------- observables

// Column sums: thread per column c of realisation r, summing p(q, c) over
// the stored rows of that column (q <= c for the triangle).
template <typename C>
__global__ void obs_cols_kernel(ObsArgs a) {
    const int64_t r = blockIdx.y;
    const RealDev rd = a.reals[r];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= rd.N) return;
    const C* psi = reinterpret_cast<const C*>(a.psi);
    const bool tri = (rd.flags & RF_TRIANGLE) != 0;
    const int qend = tri ? c + 1 : rd.rows;
    double acc = 0.0;
    for (int q = 0; q < qend; ++q) acc += prob(psi, rd, q, c);
    const double sc = a.scale[r];
    a.colsum[a.site_off[r] + c] = acc * sc * sc;
}

// Row sums: one wave per row q of realisation r (columns c >= q for the
// triangle); also records p(q, q).
template <typename C>
__global__ void obs_rows_kernel(ObsArgs a) {
    const int64_t r = blockIdx.y;
    const RealDev rd = a.reals[r];
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= rd.rows) return;
    const C* psi = reinterpret_cast<const C*>(a.psi);
    const bool tri = (rd.flags & RF_TRIANGLE) != 0;
    double acc = 0.0, dg = 0.0;
    for (int c = (tri ? q : 0) + lane; c < rd.N; c += 64) {
        const double p = prob(psi, rd, q, c);
        acc += p;
        if (c == q) dg = p;
    }
    acc = wave_sum(acc);
    dg = wave_sum(dg);
    if (lane == 0) {
        const double sc = a.scale[r];
        a.rowsum[a.site_off[r] + q] = acc * sc * sc;
        a.diag[a.site_off[r] + q] = dg * sc * sc;
    }
}

// Ensemble occupation: thread per (group, site), realisations of the group
// summed in index order (deterministic).
__global__ void obs_occ_kernel(ObsArgs a) {
    const int g = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int Ng = a.group_N[g];
    if (i >= Ng) return;
    double acc = 0.0;
    const int32_t first = a.group_first[g], last = a.group_first[g + 1];
    for (int32_t k = first; k < last; ++k) {
        const int32_t r = a.group_members[k];
        const RealDev rd = a.reals[r];
        const int64_t o = a.site_off[r] + i;
        double n;
        if (rd.rows == 1) {
            n = a.colsum[o];
        } else if (rd.flags & RF_TRIANGLE) {
            // n_i = 2 (sum_{c>=i} p(i,c) + sum_{q<=i} p(q,i)) - 2 p(i,i)
            n = 2.0 * (a.rowsum[o] + a.colsum[o]) - 2.0 * a.diag[o];
        } else {
            n = a.rowsum[o] + a.colsum[o];
        }
        acc += n;
    }
    a.out[a.group_out[g] + i] = acc / (double)(last - first);
}

// Ensemble pair correlation for two particles:
// G(i,j) = p(i,j) + p(j,i) on the full grid; 2 |phi(i,j)|^2 for bosons.
template <typename C>
__global__ void obs_pair_kernel(ObsArgs a) {
    const int g = blockIdx.z;
    const int Ng = a.group_N[g];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (i >= Ng || j >= Ng) return;
    const C* psi = reinterpret_cast<const C*>(a.psi);
    double acc = 0.0;
    const int32_t first = a.group_first[g], last = a.group_first[g + 1];
    for (int32_t k = first; k < last; ++k) {
        const int32_t r = a.group_members[k];
        const RealDev rd = a.reals[r];
        if (rd.rows == 1) continue;
        const double sc = a.scale[r];
        acc += (prob(psi, rd, i, j) + prob(psi, rd, j, i)) * sc * sc;
    }
    a.out[a.group_out[g] + Ng + (int64_t)i * Ng + j] = acc / (double)(last - first);
}

// ------------------------------------------------------------------ rescale

template <typename C>
__global__ void rescale_kernel(RescaleArgs a) {
    const int64_t r = blockIdx.y;
    const RealDev rd = a.reals[r];
    const int64_t n = (rd.flags & RF_TRIANGLE) ? (int64_t)rd.N * (rd.N + 1) / 2 : (int64_t)rd.rows * rd.N;
    const double s = a.scale[r];
    C* psi = reinterpret_cast<C*>(a.psi) + rd.state_off;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        C v = psi[i];
        v.x = v.x * s;
        v.y = v.y * s;
        psi[i] = v;
    }
}

__global__ void reset_scale_kernel(double* scale, int64_t R) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) scale[r] = 1.0;
}

}  // namespace

hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t stream) {
    if (bytes <= 0) return hipSuccess;
    if (bytes % 4) return hipErrorInvalidValue;
    const int64_t words = bytes / 4;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, hipStream_t stream) {
    const int64_t bytes = a.total * (a.dtype == 1 ? 16 : 8);
    hipError_t e = launch_fill_zero(a.psi, bytes, stream);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((a.R + 255) / 256);
    if (a.dtype == 1) hipLaunchKernelGGL(init_sites_kernel<double2>, dim3(blocks), dim3(256), 0, stream, a);
    else hipLaunchKernelGGL(init_sites_kernel<float2>, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t stream) {
    const unsigned blocks = (unsigned)((a.R + 3) / 4);   // four waves (realisations) per block
    hipLaunchKernelGGL(finalize_kernel, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_observables(const ObsArgs& a, hipStream_t stream) {
    if (a.R > 65535 || a.G > 65535 || a.max_N > 65535) return hipErrorInvalidValue;
    const dim3 gc((a.max_N + 255) / 256, (unsigned)a.R);
    const dim3 gr((a.max_N + 3) / 4, (unsigned)a.R);
    if (a.dtype == 1) {
        hipLaunchKernelGGL(obs_cols_kernel<double2>, gc, dim3(256), 0, stream, a);
        if (a.m > 1) hipLaunchKernelGGL(obs_rows_kernel<double2>, gr, dim3(256), 0, stream, a);
    } else {
        hipLaunchKernelGGL(obs_cols_kernel<float2>, gc, dim3(256), 0, stream, a);
        if (a.m > 1) hipLaunchKernelGGL(obs_rows_kernel<float2>, gr, dim3(256), 0, stream, a);
    }
    hipLaunchKernelGGL(obs_occ_kernel, dim3((a.max_N + 255) / 256, (unsigned)a.G), dim3(256), 0, stream, a);
    if (a.want_pair && a.m > 1) {
        const dim3 gp((a.max_N + 255) / 256, (unsigned)a.max_N, (unsigned)a.G);
        if (a.dtype == 1) hipLaunchKernelGGL(obs_pair_kernel<double2>, gp, dim3(256), 0, stream, a);
        else hipLaunchKernelGGL(obs_pair_kernel<float2>, gp, dim3(256), 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_rescale(const RescaleArgs& a, hipStream_t stream) {
    if (a.R > 65535) return hipErrorInvalidValue;
    const dim3 g(64, (unsigned)a.R);
    if (a.dtype == 1) hipLaunchKernelGGL(rescale_kernel<double2>, g, dim3(256), 0, stream, a);
    else hipLaunchKernelGGL(rescale_kernel<float2>, g, dim3(256), 0, stream, a);
    hipLaunchKernelGGL(reset_scale_kernel, dim3((unsigned)((a.R + 255) / 256)), dim3(256), 0, stream, a.scale, a.R);
    return hipGetLastError();
}

}  // namespace ctqw
