// Observables of three particles on a chain (the propagation is in
// step3c.hip): the two-body marginals of each realisation in FP64 and the
// ensemble occupation and pair correlation from them.
#include "ctqw_internal.hpp"

namespace ctqw {
namespace {

// Two-body marginals of realisation r: M12[x1][x2] = sum_x3 p, M13[x1][x3] =
// sum_x2 p, M23[x2][x3] = sum_x1 p (FP64, p = |psi|^2 times the load scale^2).
template <typename C>
__global__ void marg12_kernel(Obs3Args a) {
    const int r = blockIdx.z;
    const RealDev rd = a.reals[r];
    const int N = rd.N;
    const int lane = threadIdx.x & 63;
    const int x2 = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int x1 = blockIdx.y;
    if (x2 >= N) return;
    const C* psi = reinterpret_cast<const C*>(a.psi) + rd.state_off + ((int64_t)x1 * N + x2) * N;
    double acc = 0.0;
    for (int x3 = lane; x3 < N; x3 += 64) {
        const C v = psi[x3];
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) {
        const double sc = a.scale[r];
        a.M[(int64_t)r * 3 * N * N + (int64_t)x1 * N + x2] = acc * sc * sc;
    }
}

template <typename C>
__global__ void marg13_23_kernel(Obs3Args a) {
    const int r = blockIdx.z;
    const RealDev rd = a.reals[r];
    const int N = rd.N;
    const int x3 = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;   // x1 for M13, x2 for M23
    if (x3 >= N) return;
    const C* psi = reinterpret_cast<const C*>(a.psi) + rd.state_off;
    const int64_t NN = (int64_t)N * N;
    double s13 = 0.0, s23 = 0.0;
    for (int k = 0; k < N; ++k) {
        const C u = psi[(int64_t)y * NN + (int64_t)k * N + x3];    // x1 = y, x2 = k
        s13 += (double)u.x * u.x + (double)u.y * u.y;
        const C v = psi[(int64_t)k * NN + (int64_t)y * N + x3];    // x1 = k, x2 = y
        s23 += (double)v.x * v.x + (double)v.y * v.y;
    }
    const double sc = a.scale[r];
    double* M = a.M + (int64_t)r * 3 * NN;
    M[NN + (int64_t)y * N + x3] = s13 * sc * sc;
    M[2 * NN + (int64_t)y * N + x3] = s23 * sc * sc;
}

// Ensemble over the realisations of a group (index order):
//   occupation n(i) = sum_j M12[i][j] + M12[j][i] + M13[j][i]
//   pair G(i,j) = M12 + M12^T + M13 + M13^T + M23 + M23^T at (i, j).
__global__ void obs3_ensemble_kernel(Obs3Args a) {
    const int g = blockIdx.z;
    const int N = a.group_N[g];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (i >= N || j >= N) return;
    const int64_t NN = (int64_t)N * N;
    const int32_t first = a.group_first[g], last = a.group_first[g + 1];
    double occ = 0.0, pair = 0.0;
    for (int32_t k = first; k < last; ++k) {
        const int32_t r = a.group_members[k];
        const double* M = a.M + (int64_t)r * 3 * NN;
        const double* M12 = M;
        const double* M13 = M + NN;
        const double* M23 = M + 2 * NN;
        const int64_t ij = (int64_t)i * N + j, ji = (int64_t)j * N + i;
        occ += M12[ij] + M12[ji] + M13[ji];
        pair += M12[ij] + M12[ji] + M13[ij] + M13[ji] + M23[ij] + M23[ji];
    }
    const double inv = 1.0 / (double)(last - first);
    // occupation: thread (i, j) holds the j-th term of n(i); reduce over j in order
    a.occ_terms[(int64_t)g * NN + (int64_t)i * N + j] = occ * inv;
    if (a.want_pair) a.out[a.group_out[g] + N + (int64_t)i * N + j] = pair * inv;
}

__global__ void obs3_occ_kernel(Obs3Args a) {
    const int g = blockIdx.y;
    const int N = a.group_N[g];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t NN = (int64_t)N * N;
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += a.occ_terms[(int64_t)g * NN + (int64_t)i * N + j];
    a.out[a.group_out[g] + i] = s;
}

}  // namespace

hipError_t launch_obs3(const Obs3Args& a, int dtype, hipStream_t s) {
    if (a.R > 65535 || a.max_N > 65535 || a.G > 65535) return hipErrorInvalidValue;
    const int N = a.max_N;
    if (dtype == 1) {
        hipLaunchKernelGGL(marg12_kernel<double2>, dim3((N + 3) / 4, N, (unsigned)a.R), dim3(256), 0, s, a);
        hipLaunchKernelGGL(marg13_23_kernel<double2>, dim3((N + 255) / 256, N, (unsigned)a.R), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL(marg12_kernel<float2>, dim3((N + 3) / 4, N, (unsigned)a.R), dim3(256), 0, s, a);
        hipLaunchKernelGGL(marg13_23_kernel<float2>, dim3((N + 255) / 256, N, (unsigned)a.R), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(obs3_ensemble_kernel, dim3((N + 255) / 256, N, (unsigned)a.G), dim3(256), 0, s, a);
    hipLaunchKernelGGL(obs3_occ_kernel, dim3((N + 255) / 256, (unsigned)a.G), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ctqw
