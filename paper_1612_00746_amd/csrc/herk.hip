// Hermitian rank-R update of the ensemble-averaged density matrix (Eq. 2),
//     rho = (1/R) sum_r |a_r><a_r| = A A^H / R,   A: D x R complex,
// on the matrix cores, lower triangle only.  The paper forms rho with one
// rank-1 update per realisation; here the R rank-1 updates are one
// contraction over r.
//
// With a = ar + i ai, a product term a_i conj(a_j) is
//     Re = ar_i ar_j + ai_i ai_j,      Im = ai_i ar_j - ar_i ai_j,
// i.e. two real inner products of length 2 per realisation: the real and
// imaginary parts of one complex entry are the two k-slots of one MFMA
// step.  For complex64, v_mfma_f32_32x32x2_f32 takes, per lane l, the
// A entry of row l % 32 and k-slot l / 32, and the B entry of the same
// k-slot and column l % 32: with A = (ar_i, ai_i) and B = (ar_j, ai_j) it
// accumulates Re; with A' = (ai_i, -ar_i) and the same B, Im.  For
// complex128, v_mfma_f64_16x16x4_f64 takes four k-slots: two complex
// realisations per step.
//
// Input: the group's gathered states in split planes [re / im][Rp][Dp]
// (realisation-major, each realisation's D entries contiguous, zero padding
// up to Dp rows and Rp realisations), so that every tile and stage is
// loaded without bounds tests.  Work item: one tile of the lower triangle.
// The product is formed for the transposed tile -- MFMA rows from the
// tile's column block, MFMA columns from its row block -- so that each
// lane's accumulators hold consecutive rows of rho in column-major order
// and the conjugated values are stored 256 contiguous bytes per half-wave.
// Tiles on the diagonal store only their lower part; diagonal entries are
// stored with imaginary part 0 (rho is Hermitian).
#include "density.hpp"

namespace ctqw {
namespace herk_detail {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Tile index t -> (P, Q), P >= Q, row-major over the lower triangle.
__device__ __forceinline__ void tile_of(int64_t t, int* P, int* Q) {
    int p = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(p + 1) * (p + 2) / 2 <= t) ++p;
    while ((int64_t)p * (p + 1) / 2 > t) --p;
    *P = p;
    *Q = (int)(t - (int64_t)p * (p + 1) / 2);
}

// complex64: block tile 128 x 128, 4 waves of 64 x 64 (2 x 2 MFMA blocks of
// 32 x 32), stages of KC = 16 realisations staged in LDS, double-buffered.
constexpr int TS = 128;
constexpr int KC = 16;

__global__ void __launch_bounds__(256, 2) herk_c64_kernel(HerkArgs a) {
    __shared__ float lds[2][2][2][KC][TS];   // [buffer][panel: col block Q, row block P][plane][k][row]
    const int per_xcd = (int)((a.n_tiles + 7) / 8);
    const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + (blockIdx.x / 8);
    if (t >= a.n_tiles) return;   // whole block, before any barrier
    int P, Q;
    tile_of(t, &P, &Q);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;          // wave's 64 x 64 sub-tile: MFMA rows (Q side), columns (P side)
    const int64_t Dp = a.Dp, plane = (int64_t)a.Rp * Dp;
    const float* G = static_cast<const float*>(a.G);
    const int64_t q0 = (int64_t)Q * TS, p0 = (int64_t)P * TS;

    // stage loads: 2 panels x 2 planes x KC x 128 floats = 2048 float4, 8 per thread
    floatx4 st[8];
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int f = tid + 256 * u;            // [panel][plane][k][row4]
            const int panel = f >> 10, pl = (f >> 9) & 1, kk = (f >> 5) & 15, r4 = f & 31;
            const int64_t base = (panel == 0 ? q0 : p0) + 4 * r4;
            st[u] = *reinterpret_cast<const floatx4*>(G + pl * plane + (int64_t)(k0 + kk) * Dp + base);
        }
    };
    auto store_stage = [&](int b) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int f = tid + 256 * u;
            const int panel = f >> 10, pl = (f >> 9) & 1, kk = (f >> 5) & 15, r4 = f & 31;
            *reinterpret_cast<floatx4*>(&lds[b][panel][pl][kk][4 * r4]) = st[u];
        }
    };

    floatx16 accR[2][2], accI[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) accR[i][j][e] = accI[i][j][e] = 0.0f;

    const int kslot = lane >> 5;          // 0: real part, 1: imaginary part
    const int row = lane & 31;
    const float sgn = kslot ? -1.0f : 1.0f;
    const int stages = a.Rp / KC;
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int s = 0; s < stages; ++s) {
        const int b = s & 1;
        if (s + 1 < stages) load_stage((s + 1) * KC);
#pragma unroll 4
        for (int kk = 0; kk < KC; ++kk) {
            float av[2], ap[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int m = 64 * wr + 32 * i + row;
                av[i] = lds[b][0][kslot][kk][m];
                ap[i] = sgn * lds[b][0][1 - kslot][kk][m];
                const int n = 64 * wc + 32 * i + row;
                bv[i] = lds[b][1][kslot][kk][n];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    accR[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], accR[i][j], 0, 0, 0);
                    accI[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ap[i], bv[j], accI[i][j], 0, 0, 0);
                }
        }
        if (s + 1 < stages) {
            store_stage(b ^ 1);
            __syncthreads();
        }
    }

    // C'[m][n] = sum a_{Q,m} conj(a_{P,n}) = rho[Q m][P n]; rho[P n][Q m] = conj(C'[m][n]).
    // Accumulator e of a lane: MFMA row m = 8 (e / 4) + 4 (lane / 32) + e % 4, column n = lane % 32.
    const float inv = (float)a.inv_R;
    float2* rho = static_cast<float2*>(a.rho);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int m = 8 * (e >> 2) + 4 * kslot + (e & 3);
                const int64_t gc = q0 + 64 * wr + 32 * i + m;     // rho column
                const int64_t gr = p0 + 64 * wc + 32 * j + row;   // rho row
                if (gr < a.D && gc < a.D && (P != Q || gr >= gc)) {
                    float2 v;
                    v.x = accR[i][j][e] * inv;
                    v.y = gr == gc ? 0.0f : -accI[i][j][e] * inv;   // Hermitian: real diagonal
                    rho[gr + (int64_t)a.ld * gc] = v;
                }
            }
}

// complex128: block tile 64 x 64, 4 waves of 32 x 32 (2 x 2 MFMA blocks of
// 16 x 16), v_mfma_f64_16x16x4_f64 with k-slots (re, im) of two
// realisations per step; stages of 8 realisations.
constexpr int TS2 = 64;
constexpr int KC2 = 8;

__global__ void __launch_bounds__(256, 2) herk_c128_kernel(HerkArgs a) {
    __shared__ double lds[2][2][2][KC2][TS2];   // [buffer][panel][plane][k][row]
    const int per_xcd = (int)((a.n_tiles + 7) / 8);
    const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + (blockIdx.x / 8);
    if (t >= a.n_tiles) return;
    int P, Q;
    tile_of(t, &P, &Q);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int64_t Dp = a.Dp, plane = (int64_t)a.Rp * Dp;
    const double* G = static_cast<const double*>(a.G);
    const int64_t q0 = (int64_t)Q * TS2, p0 = (int64_t)P * TS2;

    // stage: 2 panels x 2 planes x 8 x 64 doubles = 2048 doubles = 1024 double2, 4 per thread
    typedef double doublex2 __attribute__((ext_vector_type(2)));
    doublex2 st[4];
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int f = tid + 256 * u;            // [panel][plane][k][row2]
            const int panel = f >> 9, pl = (f >> 8) & 1, kk = (f >> 5) & 7, r2 = f & 31;
            const int64_t base = (panel == 0 ? q0 : p0) + 2 * r2;
            st[u] = *reinterpret_cast<const doublex2*>(G + pl * plane + (int64_t)(k0 + kk) * Dp + base);
        }
    };
    auto store_stage = [&](int b) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int f = tid + 256 * u;
            const int panel = f >> 9, pl = (f >> 8) & 1, kk = (f >> 5) & 7, r2 = f & 31;
            *reinterpret_cast<doublex2*>(&lds[b][panel][pl][kk][2 * r2]) = st[u];
        }
    };

    doublex4 accR[2][2], accI[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) accR[i][j][e] = accI[i][j][e] = 0.0;

    const int kslot = lane >> 4;          // 0..3: realisation kk + (kslot >> 1), part kslot & 1
    const int part = kslot & 1, sub = kslot >> 1;
    const int row = lane & 15;
    const double sgn = part ? -1.0 : 1.0;
    const int stages = a.Rp / KC2;
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int s = 0; s < stages; ++s) {
        const int b = s & 1;
        if (s + 1 < stages) load_stage((s + 1) * KC2);
#pragma unroll
        for (int kk = 0; kk < KC2; kk += 2) {
            double av[2], ap[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int m = 32 * wr + 16 * i + row;
                av[i] = lds[b][0][part][kk + sub][m];
                ap[i] = sgn * lds[b][0][1 - part][kk + sub][m];
                const int n = 32 * wc + 16 * i + row;
                bv[i] = lds[b][1][part][kk + sub][n];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], accR[i][j], 0, 0, 0);
                    accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[i], bv[j], accI[i][j], 0, 0, 0);
                }
        }
        if (s + 1 < stages) {
            store_stage(b ^ 1);
            __syncthreads();
        }
    }

    // accumulator e of a lane: MFMA row m = 4 e + lane / 16, column n = lane % 16
    const double inv = a.inv_R;
    double2* rho = static_cast<double2*>(a.rho);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = 4 * e + kslot;
                const int64_t gc = q0 + 32 * wr + 16 * i + m;
                const int64_t gr = p0 + 32 * wc + 16 * j + row;
                if (gr < a.D && gc < a.D && (P != Q || gr >= gc)) {
                    double2 v;
                    v.x = accR[i][j][e] * inv;
                    v.y = gr == gc ? 0.0 : -accI[i][j][e] * inv;    // Hermitian: real diagonal
                    rho[gr + (int64_t)a.ld * gc] = v;
                }
            }
}

}  // namespace herk_detail

int herk_tile(int dtype) { return dtype == 1 ? herk_detail::TS2 : herk_detail::TS; }
int herk_stage(int dtype) { return dtype == 1 ? herk_detail::KC2 : herk_detail::KC; }

hipError_t launch_herk(const HerkArgs& a, int dtype, hipStream_t s) {
    if (a.n_tiles <= 0) return hipSuccess;
    const int64_t blocks = ((a.n_tiles + 7) / 8) * 8;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    if (dtype == 1)
        hipLaunchKernelGGL(herk_detail::herk_c128_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(herk_detail::herk_c64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ctqw
