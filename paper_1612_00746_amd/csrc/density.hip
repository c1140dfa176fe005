// Ensemble-averaged density matrix of one lattice-size group (Eq. 2):
//   rho = (1/R_g) sum_{r in g} |psi_r><psi_r|,
// in the basis of the state layout (bosons and fermions: the triangle basis,
// whose coefficients are sqrt(2) phi off the diagonal).  The group's states
// are gathered into split real / imaginary planes (load scale and basis
// weights applied, zero padding to whole tiles and stages), the lower
// triangle of rho = A A^H / R_g is formed on the matrix cores (herk.hip),
// and a last kernel mirrors it when the full matrix is asked for.
#include "density.hpp"

#include <algorithm>

namespace ctqw {
namespace {

template <typename C>
__global__ void gather_group_kernel(DensityArgs a) {
    using T = decltype(C{}.x);
    const int64_t k = blockIdx.y;   // member index in the group (padded)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.Dp) return;
    T* re = reinterpret_cast<T*>(a.A) + k * a.Dp + i;
    T* im = re + a.Rp * a.Dp;
    if (i >= a.D || k >= a.R_g) {
        *re = T(0);
        *im = T(0);
        return;
    }
    const int32_t r = a.members[k];
    const RealDev rd = a.reals[r];
    const C* psi = reinterpret_cast<const C*>(a.psi) + rd.state_off;
    double w = a.scale[r];
    if (a.triangle) {
        // row-major upper triangle: find (x1, x2) of i to tell the diagonal
        const int N = rd.N;
        int x1 = (int)((2.0 * N + 1.0 - sqrt((2.0 * N + 1.0) * (2.0 * N + 1.0) - 8.0 * (double)i)) / 2.0);
        while (x1 > 0 && (int64_t)x1 * N - ((int64_t)x1 * (x1 - 1)) / 2 > i) --x1;
        while ((int64_t)(x1 + 1) * N - ((int64_t)(x1 + 1) * x1) / 2 <= i) ++x1;
        const int64_t row0 = (int64_t)x1 * N - ((int64_t)x1 * (x1 - 1)) / 2;
        const int x2 = x1 + (int)(i - row0);
        if (x2 != x1) w *= 1.4142135623730950488;
    }
    const C v = psi[i];
    *re = static_cast<T>(v.x * w);
    *im = static_cast<T>(v.y * w);
}

// rho[j][i] = conj(rho[i][j]) for i > j (column-major, ld): the upper
// triangle from the lower, one 32 x 32 tile pair per block iteration.  The
// block reads lower tile (bi, bj), bi >= bj, down its columns (coalesced),
// and writes its conjugate transpose into upper tile (bj, bi), again down
// the columns, through a padded LDS tile.  Only strictly lower elements are
// copied, so on a diagonal tile the elements read and the elements written
// are disjoint.  Block rows of tiles bi = blockIdx.x; tile columns strided
// over the grid's second dimension; blocks with bj > bi have nothing to do.
template <typename C>
__global__ __launch_bounds__(256) void mirror_kernel(void* rho, int64_t D, int64_t ld) {
    __shared__ C tile[32][33];
    C* m = reinterpret_cast<C*>(rho);
    const int tx = (int)(threadIdx.x & 31), ty = (int)(threadIdx.x >> 5);
    const int64_t bi = blockIdx.x;
    for (int64_t bj = blockIdx.y; bj <= bi; bj += gridDim.y) {
        const int64_t i = bi * 32 + tx;            // source row
        for (int k = 0; k < 32; k += 8) {
            const int64_t j = bj * 32 + ty + k;    // source column
            if (i < D && j < i) tile[ty + k][tx] = m[i + ld * j];
        }
        __syncthreads();
        const int64_t jj = bj * 32 + tx;           // destination row (source column)
        for (int k = 0; k < 32; k += 8) {
            const int64_t ii = bi * 32 + ty + k;   // destination column (source row)
            if (ii < D && jj < ii) {
                C v = tile[tx][ty + k];
                v.y = -v.y;
                m[jj + ld * ii] = v;
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_density_gather(const DensityArgs& a, int dtype, hipStream_t s) {
    if (a.R_g <= 0 || a.Rp > 65535 || a.Rp < a.R_g || a.Dp < a.D) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.Dp + 255) / 256), (unsigned)a.Rp);
    if (dtype == 1)
        hipLaunchKernelGGL(gather_group_kernel<double2>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(gather_group_kernel<float2>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_density_mirror(void* rho, int64_t D, int64_t ld, int dtype, hipStream_t s) {
    if (D > 2147483647) return hipErrorInvalidValue;
    const int64_t tiles = (D + 31) / 32;
    const dim3 grid((unsigned)tiles, (unsigned)std::min<int64_t>(tiles, 65535));
    if (dtype == 1)
        hipLaunchKernelGGL(mirror_kernel<double2>, grid, dim3(256), 0, s, rho, D, ld);
    else
        hipLaunchKernelGGL(mirror_kernel<float2>, grid, dim3(256), 0, s, rho, D, ld);
    return hipGetLastError();
}

}  // namespace ctqw
