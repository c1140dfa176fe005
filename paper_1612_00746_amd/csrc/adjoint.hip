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
// The levels -- the forward vectors v_i and the Horner chain, each Horner
// level contracting its input u_L with v_L while it forms u_(L-1) (lambda_k
// at L = 0) -- run in passes of several levels (adjoint_pipe_impl.hpp).
// This file holds the loss weights (lambda and the loss from the final
// state) and the reduction of the per-realisation sums into the gradient.
#include "adjoint_common.hpp"

namespace ctqw {
namespace {

using namespace adj;

__device__ __forceinline__ int64_t index_of(const RealDev& rd, int q, int c) {
    if (rd.flags & RF_TRIANGLE) {
        const int a = q < c ? q : c, b = q < c ? c : q;
        return (int64_t)a * rd.N - ((int64_t)a * (a + 1)) / 2 + b;
    }
    return (int64_t)q * rd.N + c;
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

// Sum over realisations of the per-realisation gradients:
// out_J[b] = 2 dt sum_r (gJ[r][b] + sum_w gV[r][w][b]) (the column part, then
// the row parts of the bands in band order), out_E likewise with gE, gR; and
// the loss (1/R) sum_r sum_q row_loss[r][q].  Block b < N: site b, thread t
// summing realisations t, t + 256, ... in order, then a fixed tree over the
// threads (deterministic).  Block N: the loss, the same way.
__global__ void __launch_bounds__(256) adj_reduce_kernel(AdjReduceArgs a) {
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    __shared__ double red[2][256];
    double s0 = 0.0, s1 = 0.0;
    if (b < a.N) {
        for (int64_t r = t; r < a.R; r += 256) {
            const int64_t o = a.site_off[r] + b;
            double vj = 0.0, ve = 0.0;
            for (int w = 0; w < a.nb; ++w) {
                vj += a.gV[(r * a.nb + w) * a.row_stride + b];
                ve += a.gR[(r * a.nb + w) * a.row_stride + b];
            }
            s0 += a.gJ[o] + vj;
            s1 += a.gE[o] + ve;
        }
    } else {
        for (int64_t r = t; r < a.R; r += 256) {
            double lr = 0.0;
            for (int q = 0; q < a.rows; ++q) lr += a.row_loss[a.site_off[r] + q];
            s0 += lr;
        }
    }
    red[0][t] = s0;
    red[1][t] = s1;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (t < k) {
            red[0][t] += red[0][t + k];
            red[1][t] += red[1][t + k];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (b < a.N) {
            a.out[b] = 2.0 * a.dt * red[0][0];
            a.out[a.N + b] = 2.0 * a.dt * red[1][0];
        } else {
            a.out[2 * a.N] = red[0][0] / (double)a.R;
        }
    }
}

}  // namespace

hipError_t launch_adj_weights(const AdjWeightArgs& a, hipStream_t s) {
    if (a.R > 65535) return hipErrorInvalidValue;
    const dim3 g((unsigned)a.max_rows, (unsigned)a.R);
    if (a.dtype == 1) hipLaunchKernelGGL(weights_kernel<double2>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(weights_kernel<float2>, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_reduce(const AdjReduceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(adj_reduce_kernel, dim3((unsigned)a.N + 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ctqw
