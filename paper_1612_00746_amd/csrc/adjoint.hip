// Kernels of the discrete adjoint of the truncated-Taylor step.
//
// One step is psi_{k+1} = p(A) psi_k with A = -i dt H and p(z) = sum_{j<=n}
// z^j / j! (Alg. 3 / Eqs. 6-7).  For a loss L(psi_T) with adjoint state
// lambda = dL/d(conj psi), the step's contribution to dL/dtheta is
//     2 Re sum_{i<n} < u_i | dA/dtheta | v_i >,   v_i = A^i psi_k,
// where u_{n-1} = lambda/n!,  u_i = lambda/(i+1)! + A^dagger u_{i+1}  (Horner),
// and lambda_k = p(A)^dagger lambda_{k+1} = lambda_{k+1} + A^dagger u_0.  H is
// real symmetric (equal rates both ways, Sec. 2.2), so A^dagger = +i dt H:
// the same stencil with the opposite sign.  dA/dtheta = -i dt dH/dtheta, so
// the contribution is 2 dt Im <u_i | dH/dtheta | v_i>.
//
// The kernels work on the whole batch: `apply_kernel` computes
// y = s (-i) (dt H) x + c z for every stored amplitude (s = +1 for A, -1 for
// A^dagger); `contract_*` accumulate Im <u| E |v> for every bond operator E
// (hopping across one bond for every particle) and every site operator (the
// occupation of one node) into per-realisation FP64 sums.  Bosons are stored
// as the symmetric function on x1 <= x2 and read with mirrored indices, so
// all inner products are full-grid inner products.
#include "ctqw_internal.hpp"

namespace ctqw {
namespace {

__device__ __forceinline__ int wrapi(int x, int n) { int r = x % n; return r < 0 ? r + n : r; }

__device__ __forceinline__ int64_t index_of(const RealDev& rd, int q, int c) {
    if (rd.flags & RF_TRIANGLE) {
        const int a = q < c ? q : c, b = q < c ? c : q;
        return (int64_t)a * rd.N - ((int64_t)a * (a + 1)) / 2 + b;
    }
    return (int64_t)q * rd.N + c;
}

template <typename C>
__device__ __forceinline__ C ld(const C* __restrict__ base, const RealDev& rd, int q, int c) {
    return base[rd.state_off + index_of(rd, q, c)];
}

// (dt H x)(q, c) with the dt-scaled tables of the step kernel.
template <typename T, typename C>
__device__ __forceinline__ void apply_h(const C* __restrict__ x, const RealDev& rd, const T* __restrict__ Jt,
                                        const T* __restrict__ Et, T Udt, int q, int c, T& hr, T& hi) {
    const int N = rd.N, rows = rd.rows;
    const bool periodic = (rd.flags & RF_PERIODIC) != 0;
    const T* Jc = Jt + rd.param_off;
    const T* Ec = Et + rd.param_off;
    const T* Jr = Jt + rd.row_param_off;
    const T* Er = Et + rd.row_param_off;
    const C s = ld(x, rd, q, c);
    T d = Er[q] + Ec[c];
    if (rows > 1) {
        int dd = q - c;
        dd = dd < 0 ? -dd : dd;
        if (periodic && N - dd < dd) dd = N - dd;
        if (dd == ((rd.flags & RF_NEAREST) ? 1 : 0)) d += Udt;
    }
    hr = d * s.x;
    hi = d * s.y;
    // column neighbours (bond c-1 joins c-1 and c, bond c joins c and c+1)
    if (c > 0 || periodic) {
        const int cl = c > 0 ? c - 1 : N - 1;
        const C v = ld(x, rd, q, cl);
        const T j = Jc[cl];
        hr += j * v.x;
        hi += j * v.y;
    }
    if (c < N - 1 || periodic) {
        const int cr = c < N - 1 ? c + 1 : 0;
        const C v = ld(x, rd, q, cr);
        const T j = Jc[c];
        hr += j * v.x;
        hi += j * v.y;
    }
    if (rows > 1) {
        if (q > 0 || periodic) {
            const int qu = q > 0 ? q - 1 : rows - 1;
            const C v = ld(x, rd, qu, c);
            const T j = Jr[qu];
            hr += j * v.x;
            hi += j * v.y;
        }
        if (q < rows - 1 || periodic) {
            const int qd = q < rows - 1 ? q + 1 : 0;
            const C v = ld(x, rd, qd, c);
            const T j = Jr[q];
            hr += j * v.x;
            hi += j * v.y;
        }
    }
}

// y = s * (-i) * (dt H x) + cz * z  over every stored amplitude; x may be
// null (then only cz * z), z may be null (cz ignored).
template <typename T>
__global__ void apply_kernel(AdjApplyArgs a) {
    using C = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    const int r = blockIdx.z;
    const RealDev rd = a.reals[r];
    const int q = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rd.rows || c >= rd.N) return;
    if ((rd.flags & RF_TRIANGLE) && c < q) return;
    const C* x = reinterpret_cast<const C*>(a.x);
    const C* z = reinterpret_cast<const C*>(a.z);
    C* y = reinterpret_cast<C*>(a.y);
    T yr = T(0), yi = T(0);
    if (x) {
        T hr, hi;
        apply_h<T, C>(x, rd, reinterpret_cast<const T*>(a.Jt), reinterpret_cast<const T*>(a.Et),
                      static_cast<T>(rd.U * a.dt), q, c, hr, hi);
        // s (-i)(hr + i hi) = s (hi - i hr)
        const T sg = static_cast<T>(a.sign);
        yr = sg * hi;
        yi = -sg * hr;
    }
    const int64_t o = rd.state_off + index_of(rd, q, c);
    if (z) {
        const C zv = z[o];
        const T cz = static_cast<T>(a.cz);
        yr += cz * zv.x;
        yi += cz * zv.y;
    }
    C out;
    out.x = yr;
    out.y = yi;
    y[o] = out;
}

// Im( conj(u) v ) in FP64.
template <typename C>
__device__ __forceinline__ double im_uv(const C& u, const C& v) {
    return (double)u.x * (double)v.y - (double)u.y * (double)v.x;
}

// Column parts: thread per column b of realisation r, summing over all rows
//   bond b: Im conj(u(q,b)) v(q,b+1) + Im conj(u(q,b+1)) v(q,b)
//   site b: Im conj(u(q,b)) v(q,b)
// (the only parts for one particle; doubled for the symmetric boson function).
template <typename C>
__global__ void contract_cols_kernel(AdjContractArgs a) {
    const int r = blockIdx.y;
    const RealDev rd = a.reals[r];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= rd.N) return;
    const C* u = reinterpret_cast<const C*>(a.u);
    const C* v = reinterpret_cast<const C*>(a.v);
    const bool periodic = (rd.flags & RF_PERIODIC) != 0;
    const bool has_bond = periodic || b < rd.N - 1;
    const int b1 = b + 1 < rd.N ? b + 1 : 0;
    double sb = 0.0, ss = 0.0;
    for (int q = 0; q < rd.rows; ++q) {
        const C ub = ld(u, rd, q, b), vb = ld(v, rd, q, b);
        ss += im_uv(ub, vb);
        if (has_bond) {
            const C ub1 = ld(u, rd, q, b1), vb1 = ld(v, rd, q, b1);
            sb += im_uv(ub, vb1) + im_uv(ub1, vb);
        }
    }
    const double f = (rd.flags & RF_TRIANGLE) ? 2.0 : 1.0;
    const int64_t o = a.site_off[r] + b;
    a.gJ[o] += f * sb;
    a.gE[o] += f * ss;
}

// Row parts for distinguishable particles: one wave per row q,
//   bond q: sum_c Im conj(u(q,c)) v(q+1,c) + Im conj(u(q+1,c)) v(q,c)
//   site q: sum_c Im conj(u(q,c)) v(q,c)
template <typename C>
__global__ void contract_rows_kernel(AdjContractArgs a) {
    const int r = blockIdx.y;
    const RealDev rd = a.reals[r];
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= rd.rows) return;
    const C* u = reinterpret_cast<const C*>(a.u);
    const C* v = reinterpret_cast<const C*>(a.v);
    const bool periodic = (rd.flags & RF_PERIODIC) != 0;
    const bool has_bond = periodic || q < rd.rows - 1;
    const int q1 = q + 1 < rd.rows ? q + 1 : 0;
    double sb = 0.0, ss = 0.0;
    for (int c = lane; c < rd.N; c += 64) {
        const C uq = ld(u, rd, q, c), vq = ld(v, rd, q, c);
        ss += im_uv(uq, vq);
        if (has_bond) {
            const C uq1 = ld(u, rd, q1, c), vq1 = ld(v, rd, q1, c);
            sb += im_uv(uq, vq1) + im_uv(uq1, vq);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sb += __shfl_xor(sb, off, 64);
        ss += __shfl_xor(ss, off, 64);
    }
    if (lane == 0) {
        const int64_t o = a.site_off[r] + q;
        a.gJ2[o] += sb;
        a.gE2[o] += ss;
    }
}

// lambda = w(x) psi / R and the per-realisation loss sum_x w(x) |psi(x)|^2
// (full grid: off-diagonal boson entries count twice).  Block per
// (row, realisation); per-row partials are reduced in row order afterwards.
template <typename C>
__global__ void weights_kernel(AdjWeightArgs a) {
    const int r = blockIdx.y;
    const RealDev rd = a.reals[r];
    const int q = blockIdx.x;
    if (q >= rd.rows) return;
    const C* psi = reinterpret_cast<const C*>(a.psi);
    C* lam = reinterpret_cast<C*>(a.lam);
    const bool tri = (rd.flags & RF_TRIANGLE) != 0;
    const double* g = a.site_w;
    double acc = 0.0;
    for (int c = (tri ? q : 0) + threadIdx.x; c < rd.N; c += blockDim.x) {
        double w;
        if (rd.rows == 1) w = g[c];
        else if (a.kind == 0) w = g[q] + g[c];
        else w = g[q] * g[c];
        const int64_t o = rd.state_off + index_of(rd, q, c);
        const C v = psi[o];
        const double p = (double)v.x * v.x + (double)v.y * v.y;
        acc += (tri && c != q ? 2.0 : 1.0) * w * p;
        C l;
        l.x = static_cast<decltype(v.x)>(w * a.inv_R * v.x);
        l.y = static_cast<decltype(v.x)>(w * a.inv_R * v.y);
        lam[o] = l;
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.row_loss[a.site_off[r] + q] = red[0];
}

// Sum over realisations (index order) of the per-realisation gradients:
// out_J[b] = 2 dt sum_r (gJ[r][b] + gJ2[r][b]), out_E likewise; and the loss
// (1/R) sum_r sum_q row_loss[r][q].  One thread per site b (plus thread 0 of
// block 0 for the loss).
__global__ void adj_reduce_kernel(AdjReduceArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < a.N) {
        double sj = 0.0, se = 0.0;
        for (int64_t r = 0; r < a.R; ++r) {
            const int64_t o = a.site_off[r] + b;
            sj += a.gJ[o] + a.gJ2[o];
            se += a.gE[o] + a.gE2[o];
        }
        a.out[b] = 2.0 * a.dt * sj;
        a.out[a.N + b] = 2.0 * a.dt * se;
    }
    if (b == 0) {
        double l = 0.0;
        for (int64_t r = 0; r < a.R; ++r) {
            double lr = 0.0;
            for (int q = 0; q < a.rows; ++q) lr += a.row_loss[a.site_off[r] + q];
            l += lr;
        }
        a.out[2 * a.N] = l / (double)a.R;
    }
}

}  // namespace

hipError_t launch_adj_apply(const AdjApplyArgs& a, hipStream_t s) {
    if (a.R > 65535 || a.max_rows > 65535) return hipErrorInvalidValue;
    const dim3 g((a.max_N + 63) / 64, a.max_rows, (unsigned)a.R);
    if (a.dtype == 1) hipLaunchKernelGGL(apply_kernel<double>, g, dim3(64), 0, s, a);
    else hipLaunchKernelGGL(apply_kernel<float>, g, dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_contract(const AdjContractArgs& a, hipStream_t s) {
    if (a.R > 65535) return hipErrorInvalidValue;
    const dim3 gc((a.max_N + 255) / 256, (unsigned)a.R);
    const dim3 gr((a.max_rows + 3) / 4, (unsigned)a.R);
    if (a.dtype == 1) {
        hipLaunchKernelGGL(contract_cols_kernel<double2>, gc, dim3(256), 0, s, a);
        if (a.rows_part) hipLaunchKernelGGL(contract_rows_kernel<double2>, gr, dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL(contract_cols_kernel<float2>, gc, dim3(256), 0, s, a);
        if (a.rows_part) hipLaunchKernelGGL(contract_rows_kernel<float2>, gr, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_adj_weights(const AdjWeightArgs& a, hipStream_t s) {
    if (a.R > 65535) return hipErrorInvalidValue;
    const dim3 g((unsigned)a.max_rows, (unsigned)a.R);
    if (a.dtype == 1) hipLaunchKernelGGL(weights_kernel<double2>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(weights_kernel<float2>, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_reduce(const AdjReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(adj_reduce_kernel, dim3((a.N + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ctqw
