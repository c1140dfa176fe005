// One particle on a general graph (Sec. 2: node a couples to its own set of
// neighbours; a q-dimensional lattice is one such graph), R statically noisy
// realisations sharing one topology, advanced by the truncated Taylor series
// of exp(-i H dt) (Eqs. 5-7) one term per pass: term j is
//     Phi^(j) = (-i dt / j) H Phi^(j-1),   psi(t + dt) = sum_j Phi^(j),
// with H psi gathered through an ELL neighbour table.  The topology is the
// same for every realisation, the couplings and on-site energies are each
// realisation's own.  Complex128, FP64 arithmetic.
//
// Work mapping: one thread per (node, realisation); nodes along x
// (coalesced reads of the ELL slots, the couplings, the on-site energies and
// the state), realisations along y, strided over the grid's second dimension.
// Per node, term and realisation the pass reads the previous term at the
// node and its neighbours (the neighbours mostly from cache), width
// couplings and slot indices, the on-site energy and the partial sum, and
// writes the term and the partial sum: it is HBM-bound.
#include "graph.hpp"

#include <algorithm>

namespace ctqw {
namespace {

__global__ __launch_bounds__(256) void graph_term_kernel(GraphTermArgs a) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= a.n) return;
    const int64_t n = a.n;
    for (int64_t r = blockIdx.y; r < a.R; r += gridDim.y) {
        const double2* x = a.src + r * n;
        const double2 xi = x[i];
        const double e = a.onsite[r * n + i];
        double hr = e * xi.x, hi = e * xi.y;
        const double* h = a.hop + r * (int64_t)a.width * n;
        for (int32_t k = 0; k < a.width; ++k) {
            const int32_t j = a.nbr[(int64_t)k * n + i];
            if (j < 0 || j >= a.n) continue;
            const double c = h[(int64_t)k * n + i];
            const double2 xj = x[j];
            hr = fma(c, xj.x, hr);
            hi = fma(c, xj.y, hi);
        }
        // (-i c) (hr + i hi) = c hi - i c hr
        const double2 t = make_double2(a.c * hi, -a.c * hr);
        if (a.t_out) a.t_out[r * n + i] = t;
        const double2 s = a.acc_in[r * n + i];
        a.acc_out[r * n + i] = make_double2(s.x + t.x, s.y + t.y);
    }
}

// Squared FP64 norm of each realisation: block r strides over its nodes,
// then a fixed shared-memory tree, so the result does not depend on timing.
__global__ __launch_bounds__(256) void graph_norm_kernel(const double2* psi, int32_t n, double* out) {
    __shared__ double part[256];
    const int64_t r = blockIdx.x;
    const double2* x = psi + r * (int64_t)n;
    double acc = 0.0;
    for (int32_t i = (int32_t)threadIdx.x; i < n; i += 256) {
        const double2 v = x[i];
        acc = fma(v.x, v.x, fma(v.y, v.y, acc));
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = part[0];
}

}  // namespace

hipError_t launch_graph_norms(const double2* psi, int32_t n, int32_t R, double* out, hipStream_t s) {
    hipLaunchKernelGGL(graph_norm_kernel, dim3((unsigned)R), dim3(256), 0, s, psi, n, out);
    return hipGetLastError();
}

hipError_t launch_graph_term(const GraphTermArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.n + 255) / 256), (unsigned)std::min<int32_t>(a.R, 65535));
    hipLaunchKernelGGL(graph_term_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ctqw
