// Three particles on a chain: one Taylor term per pass over the state.
//
// The walk of m = 3 distinguishable particles lives on the N^3 grid
// psi[x1][x2][x3] (x3 fastest).  A time step of Alg. 3 runs n passes; pass j
// computes Phi^(j) = -(i dt / j) H Phi^(j-1) and adds it to the new state:
//   (H phi)(x) = sum_a J[x_a - 1] phi(x - e_a) + J[x_a] phi(x + e_a)
//              + (eps[x1] + eps[x2] + eps[x3] + V(x)) phi(x),
// V(x) = U * #{a < b : chain distance |x_a - x_b| == 1} (nearest neighbours)
// or U * #{a < b : x_a == x_b} (on site).  The register pipeline of the
// two-particle kernel needs a whole (x2, x3) plane per level here, which
// does not fit, so terms are not chained: the tables hold dt-scaled J, eps.
//
// Block: 64 x3 columns x 4 x2 rows; grid: (x3 blocks * x2 blocks, N, R).
// Pass 1 reads psi (scaled by the load scale), writes Phi^(1) and the sum
// psi + Phi^(1) (with a zero Kahan compensation); middle passes read
// Phi^(j-1), write Phi^(j) and update the sum; the last pass writes only the
// sum and accumulates the FP64 squared norms of the new state and of
// Phi^(n), one partial per block.
#include "ctqw_internal.hpp"

namespace ctqw {
namespace {

template <typename T> struct Cplx3;
template <> struct Cplx3<float> { using type = float2; };
template <> struct Cplx3<double> { using type = double2; };

// Non-temporal store of one amplitude: every array a pass writes is read
// again only in the next pass, after the whole state has streamed by.
template <typename C>
__device__ __forceinline__ void store_nt(C* p, C v) {
    using T = decltype(v.x);
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 x;
    x.x = v.x;
    x.y = v.y;
    __builtin_nontemporal_store(x, reinterpret_cast<v2*>(p));
}

__device__ __forceinline__ int dist(int a, int b, int N, bool periodic) {
    int d = a - b;
    d = d < 0 ? -d : d;
    if (periodic && N - d < d) d = N - d;
    return d;
}

template <typename T, bool KAHAN>
__global__ void __launch_bounds__(256) term3d_kernel(Step3Args a) {
    using C = typename Cplx3<T>::type;
    const int r = blockIdx.z;
    const RealDev rd = a.reals[r];
    const int N = rd.N;
    const int xb = (N + 63) / 64;
    const int x3 = (blockIdx.x % xb) * 64 + (threadIdx.x & 63);
    const int x2 = (blockIdx.x / xb) * 4 + (threadIdx.x >> 6);
    const int x1 = blockIdx.y;
    const bool live = x3 < N && x2 < N;
    const bool periodic = (rd.flags & RF_PERIODIC) != 0;
    const T* J = reinterpret_cast<const T*>(a.Jt) + rd.param_off;
    const T* E = reinterpret_cast<const T*>(a.Et) + rd.param_off;
    const C* in = reinterpret_cast<const C*>(a.phi_in) + rd.state_off;
    const T sc = a.first ? static_cast<T>(a.scale[r]) : T(1);
    double nrm = 0.0, tail = 0.0;
    if (live) {
        const int64_t NN = (int64_t)N * N;
        const int64_t o = (int64_t)x1 * NN + (int64_t)x2 * N + x3;
        const C s = in[o];
        T d = E[x1] + E[x2] + E[x3];
        const int want = (rd.flags & RF_NEAREST) ? 1 : 0;
        const T Udt = static_cast<T>(rd.U * a.dt);
        if (dist(x1, x2, N, periodic) == want) d += Udt;
        if (dist(x1, x3, N, periodic) == want) d += Udt;
        if (dist(x2, x3, N, periodic) == want) d += Udt;
        T hr = d * s.x, hi = d * s.y;
        // neighbours along each axis; bond b joins nodes b and b+1 (mod N on a ring)
        const int xs[3] = {x1, x2, x3};
        const int64_t st[3] = {NN, (int64_t)N, 1};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int x = xs[ax];
            if (x > 0 || periodic) {
                const int xl = x > 0 ? x - 1 : N - 1;
                const C v = in[o + (int64_t)(xl - x) * st[ax]];
                const T j = J[xl];
                hr += j * v.x;
                hi += j * v.y;
            }
            if (x < N - 1 || periodic) {
                const int xr = x < N - 1 ? x + 1 : 0;
                const C v = in[o + (int64_t)(xr - x) * st[ax]];
                const T j = J[x];
                hr += j * v.x;
                hi += j * v.y;
            }
        }
        // Phi^(j) = -(i / j) (dt H) Phi^(j-1)  (sc folds the load scale of psi)
        const T c = static_cast<T>(a.inv_j) * sc;
        const T pr = c * hi, pi = -c * hr;
        C* acc = reinterpret_cast<C*>(a.acc) + rd.state_off;
        C* cmp = reinterpret_cast<C*>(a.comp) + rd.state_off;
        C sum, cp;
        if (a.first) {
            sum.x = s.x * sc;
            sum.y = s.y * sc;
            cp.x = T(0);
            cp.y = T(0);
        } else {
            sum = acc[o];
            if (KAHAN) cp = cmp[o];
        }
        if (KAHAN) {
            const T yr = pr - cp.x, tr = sum.x + yr;
            cp.x = (tr - sum.x) - yr;
            sum.x = tr;
            const T yi = pi - cp.y, ti = sum.y + yi;
            cp.y = (ti - sum.y) - yi;
            sum.y = ti;
        } else {
            sum.x += pr;
            sum.y += pi;
        }
        store_nt(acc + o, sum);
        if (!a.last) {
            if (KAHAN) store_nt(cmp + o, cp);
            C f;
            f.x = pr;
            f.y = pi;
            store_nt(reinterpret_cast<C*>(a.phi_out) + rd.state_off + o, f);
        } else {
            nrm = (double)sum.x * sum.x + (double)sum.y * sum.y;
            tail = (double)pr * pr + (double)pi * pi;
        }
    }
    if (a.last) {
        __shared__ double red[2][256];
        red[0][threadIdx.x] = nrm;
        red[1][threadIdx.x] = tail;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                red[0][threadIdx.x] += red[0][threadIdx.x + s];
                red[1][threadIdx.x] += red[1][threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int64_t item = (int64_t)r * a.blocks_per_real + (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
            a.norm_part[item] = red[0][0];
            a.tail_part[item] = red[1][0];
        }
    }
}

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

hipError_t launch_term3d(const Step3Args& a, int kahan, int dtype, int N, hipStream_t s) {
    if (a.R > 65535 || N > 65535) return hipErrorInvalidValue;
    const int xb = (N + 63) / 64, yb = (N + 3) / 4;
    const dim3 g((unsigned)(xb * yb), (unsigned)N, (unsigned)a.R);
    if (dtype == 1) hipLaunchKernelGGL((term3d_kernel<double, false>), g, dim3(256), 0, s, a);
    else if (kahan) hipLaunchKernelGGL((term3d_kernel<float, true>), g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((term3d_kernel<float, false>), g, dim3(256), 0, s, a);
    return hipGetLastError();
}

int64_t term3d_blocks_per_real(int N) { return (int64_t)((N + 63) / 64) * ((N + 3) / 4) * N; }

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
