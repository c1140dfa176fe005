// Ensemble-averaged density matrix of one lattice-size group (Eq. 2):
//   rho = (1/R_g) sum_{r in g} |psi_r><psi_r|,
// in the basis of the state layout (bosons: the normalised symmetric basis,
// whose coefficients are sqrt(2) phi off the diagonal).  The group's states
// are gathered into a D x R_g column-major matrix A (load scale and basis
// weights applied), then rho = A A^H / R_g is one Hermitian rank-R_g update
// (a plain library contraction: rocBLAS cherk / zherk, on the matrix cores);
// a last kernel mirrors the lower triangle when the full matrix is asked for.
#include "density.hpp"

#include <rocblas/rocblas.h>

#include <algorithm>

namespace ctqw {
namespace {

template <typename C>
__global__ void gather_group_kernel(DensityArgs a) {
    const int64_t k = blockIdx.y;   // member index in the group
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.D) return;
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
    C v = psi[i];
    v.x = static_cast<decltype(v.x)>(v.x * w);
    v.y = static_cast<decltype(v.y)>(v.y * w);
    reinterpret_cast<C*>(a.A)[i + a.D * k] = v;
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
    if (a.R_g <= 0 || a.R_g > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.D + 255) / 256), (unsigned)a.R_g);
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

// rho (lower triangle) = A A^H / R_g with A: D x R_g, column-major.
int density_herk(void** handle, hipStream_t s, int dtype, int64_t D, int64_t R_g, const void* A, void* rho,
                 int64_t ld) {
    if (!*handle) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return -1;
        *handle = h;
    }
    rocblas_handle h = static_cast<rocblas_handle>(*handle);
    if (rocblas_set_stream(h, s) != rocblas_status_success) return -2;
    rocblas_status st;
    if (dtype == 1) {
        const double alpha = 1.0 / (double)R_g, beta = 0.0;
        st = rocblas_zherk(h, rocblas_fill_lower, rocblas_operation_none, (rocblas_int)D, (rocblas_int)R_g, &alpha,
                           static_cast<const rocblas_double_complex*>(A), (rocblas_int)D, &beta,
                           static_cast<rocblas_double_complex*>(rho), (rocblas_int)ld);
    } else {
        const float alpha = (float)(1.0 / (double)R_g), beta = 0.0f;
        st = rocblas_cherk(h, rocblas_fill_lower, rocblas_operation_none, (rocblas_int)D, (rocblas_int)R_g, &alpha,
                           static_cast<const rocblas_float_complex*>(A), (rocblas_int)D, &beta,
                           static_cast<rocblas_float_complex*>(rho), (rocblas_int)ld);
    }
    return st == rocblas_status_success ? 0 : (int)st;
}

void density_release(void* handle) {
    if (handle) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(handle));
}

}  // namespace ctqw
