// Fused stencil + truncated-Taylor step for one and two particles on a chain.
//
// One step of Alg. 3 (Eqs. 6-7): Phi^(0) = psi, Phi^(j) = -(i dt / j) H Phi^(j-1),
// psi(t + dt) = sum_{j<=n} Phi^(j), with H applied matrix-free:
//   (H phi)(q, c) = J[q-1] phi(q-1, c) + J[q] phi(q+1, c)
//                 + J[c-1] phi(q, c-1) + J[c] phi(q, c+1)
//                 + (eps[q] + eps[c] + V(q, c)) phi(q, c)
// (Eq. 1 with the Kronecker-sum structure of m = 2 particles; one particle is
// the single-row case).  The paper builds H from a reduced matrix and a shared
// topology matrix (Sec. 2.2) and runs one kernel per term with device-wide
// copies in between; here all n terms of a step are chained in registers
// during one pass over the state:
//
//  * a wave owns a band of 64*P consecutive columns (P per lane, so global
//    loads and stores of a row are contiguous) and sweeps the rows;
//  * a pipeline of n levels runs down the rows: at sweep iteration i, level 0
//    loads row i, level j works on row i - j from level j-1 on rows i-j-1,
//    i-j, i-j+1 (all already in registers), and row i - n is complete and
//    stored.  Each level keeps a three-row window; the partial sums of the
//    rows in flight (and the separate sums of their terms) sit in an (n+1)-row
//    window.  Windows start at zero and rows outside the sweep stay zero, so
//    the pipeline fills and drains without per-level tests (the bond above
//    the first row and below the last row of an open chain is 0).
//  * the coefficients are pre-scaled by dt on the host and the recursion
//    carries Psi_j = (-i dt H)^j psi = j! Phi^(j): the -i is a swap of the
//    real and imaginary parts and the 1/j! multiplies the term as it is
//    added, so a level costs the stencil plus the accumulation.
//  * column neighbours come from the adjacent lanes through DPP row shifts
//    (wave_shr / wave_shl); the band overlaps its neighbours by n columns
//    (the halo), recomputed by both.
//  * HBM traffic per step: each amplitude is read once and written once.
//
// Two bosons are stored as the symmetric function phi(x1, x2) on x1 <= x2,
// row-major: the diagonal uses the mirrored neighbours phi(q, q-1) =
// phi(q-1, q) and phi(q+1, q) = phi(q, q+1), i.e. doubled couplings to the
// row above and the column to the right, with the lower triangle held at 0.
// Two fermions (open chain) use the same layout for the antisymmetric
// phi: the diagonal is held at 0 as well, and since every neighbour of an
// element above it that lies across the diagonal is a diagonal element,
// no coupling changes.
//
// Complex64 state can sum the terms j >= 1 apart from psi and add them to it
// once per step (compensated accumulation: one rounding of the state per
// step instead of one per term).  The squared norm of the new state and of
// the last term are accumulated in FP64 per item (the paper checks the norm
// every step, Alg. 3).
#pragma once
#include "ctqw_internal.hpp"

namespace ctqw {
namespace step2d_detail {

template <typename T> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };

// Lane i receives lane i-1 (lane 0 receives 0).
__device__ __forceinline__ float from_left(float x) {
    return __builtin_amdgcn_update_dpp(0.0f, x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ double from_left(double x) {
    return __builtin_amdgcn_update_dpp(0.0, x, 0x138, 0xF, 0xF, true);
}
// Lane i receives lane i+1 (lane 63 receives 0).
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float from_right(float x) {
    return __builtin_amdgcn_update_dpp(0.0f, x, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ double from_right(double x) {
    return __builtin_amdgcn_update_dpp(0.0, x, 0x130, 0xF, 0xF, true);
}

// The complex64 full-grid stencil of one level, h = (H Psi) scaled by dt:
//   h(c) = d(c) m(c) + Ju u(c) + Jd v(c) + jl(c) m(c-1) + jr(c) m(c+1)
// (m, u, v: the level below on this row and the rows above and below; Ju,
// Jd: the wave-uniform row bonds), accumulated in this order, real and
// imaginary parts alike.  Written out so that the neighbour columns held
// by the adjacent lanes enter through DPP-routed FMAs (no separate moves)
// and the independent chains are interleaved.  A DPP read of a VGPR must
// follow the VALU write of that register by two wait states; every DPP
// instruction here comes after at least six VALU instructions of the same
// block, and its source is an input of the block.
__device__ __forceinline__ void stencil_c64_p1(float& hr, float& hi, float d, float mr, float mi, float ur, float ui,
                                               float vr, float vi, float Ju, float Jd, float jl, float jr) {
    asm("v_mul_f32 %0, %2, %3\n\t"
        "v_mul_f32 %1, %2, %4\n\t"
        "v_fmac_f32 %0, %9, %5\n\t"
        "v_fmac_f32 %1, %9, %6\n\t"
        "v_fmac_f32 %0, %10, %7\n\t"
        "v_fmac_f32 %1, %10, %8\n\t"
        "v_fmac_f32_dpp %0, %3, %11 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %4, %11 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %0, %3, %12 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %4, %12 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(hr), "=&v"(hi)
        : "v"(d), "v"(mr), "v"(mi), "v"(ur), "v"(ui), "v"(vr), "v"(vi), "s"(Ju), "s"(Jd), "v"(jl), "v"(jr));
}
// Two columns per lane: column 0's left neighbour and column 1's right
// neighbour come from the adjacent lanes, the others from this lane.
__device__ __forceinline__ void stencil_c64_p2(float (&hr)[2], float (&hi)[2], const float (&d)[2], const float (&mr)[2],
                                               const float (&mi)[2], const float (&ur)[2], const float (&ui)[2],
                                               const float (&vr)[2], const float (&vi)[2], float Ju, float Jd,
                                               const float (&jl)[2], const float (&jr)[2]) {
    asm("v_mul_f32 %0, %4, %6\n\t"
        "v_mul_f32 %1, %4, %7\n\t"
        "v_mul_f32 %2, %5, %8\n\t"
        "v_mul_f32 %3, %5, %9\n\t"
        "v_fmac_f32 %0, %18, %10\n\t"
        "v_fmac_f32 %1, %18, %11\n\t"
        "v_fmac_f32 %2, %18, %12\n\t"
        "v_fmac_f32 %3, %18, %13\n\t"
        "v_fmac_f32 %0, %19, %14\n\t"
        "v_fmac_f32 %1, %19, %15\n\t"
        "v_fmac_f32 %2, %19, %16\n\t"
        "v_fmac_f32 %3, %19, %17\n\t"
        "v_fmac_f32_dpp %0, %8, %20 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %9, %20 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32 %2, %21, %6\n\t"
        "v_fmac_f32 %3, %21, %7\n\t"
        "v_fmac_f32 %0, %22, %8\n\t"
        "v_fmac_f32 %1, %22, %9\n\t"
        "v_fmac_f32_dpp %2, %6, %23 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %3, %7, %23 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(hr[0]), "=&v"(hi[0]), "=&v"(hr[1]), "=&v"(hi[1])
        : "v"(d[0]), "v"(d[1]), "v"(mr[0]), "v"(mi[0]), "v"(mr[1]), "v"(mi[1]), "v"(ur[0]), "v"(ui[0]), "v"(ur[1]),
          "v"(ui[1]), "v"(vr[0]), "v"(vi[0]), "v"(vr[1]), "v"(vi[1]), "s"(Ju), "s"(Jd), "v"(jl[0]), "v"(jl[1]),
          "v"(jr[0]), "v"(jr[1]));
}

// The same stencils without the diagonal product, for rows where the
// diagonal of H is zero on every lane (no on-site energies, no interacting
// column in the band): the sum starts from the bond above.  The DPP reads
// come after four or eight VALU instructions of the block.
__device__ __forceinline__ void stencil_c64_p1_nd(float& hr, float& hi, float mr, float mi, float ur, float ui,
                                                  float vr, float vi, float Ju, float Jd, float jl, float jr) {
    asm("v_mul_f32 %0, %8, %4\n\t"
        "v_mul_f32 %1, %8, %5\n\t"
        "v_fmac_f32 %0, %9, %6\n\t"
        "v_fmac_f32 %1, %9, %7\n\t"
        "v_fmac_f32_dpp %0, %2, %10 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %3, %10 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %0, %2, %11 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %3, %11 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(hr), "=&v"(hi)
        : "v"(mr), "v"(mi), "v"(ur), "v"(ui), "v"(vr), "v"(vi), "s"(Ju), "s"(Jd), "v"(jl), "v"(jr));
}
__device__ __forceinline__ void stencil_c64_p2_nd(float (&hr)[2], float (&hi)[2], const float (&mr)[2],
                                                  const float (&mi)[2], const float (&ur)[2], const float (&ui)[2],
                                                  const float (&vr)[2], const float (&vi)[2], float Ju, float Jd,
                                                  const float (&jl)[2], const float (&jr)[2]) {
    asm("v_mul_f32 %0, %16, %8\n\t"
        "v_mul_f32 %1, %16, %9\n\t"
        "v_mul_f32 %2, %16, %10\n\t"
        "v_mul_f32 %3, %16, %11\n\t"
        "v_fmac_f32 %0, %17, %12\n\t"
        "v_fmac_f32 %1, %17, %13\n\t"
        "v_fmac_f32 %2, %17, %14\n\t"
        "v_fmac_f32 %3, %17, %15\n\t"
        "v_fmac_f32_dpp %0, %6, %18 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %7, %18 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32 %2, %19, %4\n\t"
        "v_fmac_f32 %3, %19, %5\n\t"
        "v_fmac_f32 %0, %20, %6\n\t"
        "v_fmac_f32 %1, %20, %7\n\t"
        "v_fmac_f32_dpp %2, %4, %21 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %3, %5, %21 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(hr[0]), "=&v"(hi[0]), "=&v"(hr[1]), "=&v"(hi[1])
        : "v"(mr[0]), "v"(mi[0]), "v"(mr[1]), "v"(mi[1]), "v"(ur[0]), "v"(ui[0]), "v"(ur[1]), "v"(ui[1]),
          "v"(vr[0]), "v"(vi[0]), "v"(vr[1]), "v"(vi[1]), "s"(Ju), "s"(Jd), "v"(jl[0]), "v"(jl[1]), "v"(jr[0]),
          "v"(jr[1]));
}

// Raw buffer resources: the last descriptor word for gfx9-family buffers
// without format conversion.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufferWord3 = 0x00020000;
// Cache policy of the state's stores: non-temporal (the new state is read
// again only at the next step, after the whole state has streamed through
// the caches).  Loads keep the default policy: the halo columns of adjacent
// bands are read twice.
constexpr int kStorePolicy = 2;   // nt
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename C>
__device__ __forceinline__ C buffer_load_cplx(__amdgpu_buffer_rsrc_t rs, uint32_t off);
template <>
__device__ __forceinline__ float2 buffer_load_cplx<float2>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
template <>
__device__ __forceinline__ double2 buffer_load_cplx<double2>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    return make_double2(__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z));
}
__device__ __forceinline__ void buffer_store_cplx(float2 c, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x2 v;
    v.x = __float_as_uint(c.x);
    v.y = __float_as_uint(c.y);
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, (int)off, 0, kStorePolicy);
}
__device__ __forceinline__ void buffer_store_cplx(double2 c, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x4 v;
    v.x = (unsigned)__double2loint(c.x);
    v.y = (unsigned)__double2hiint(c.x);
    v.z = (unsigned)__double2loint(c.y);
    v.w = (unsigned)__double2hiint(c.y);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, kStorePolicy);
}

__host__ __device__ constexpr int window_rows(int nt) { return ((nt + 3) / 3) * 3; }
__host__ __device__ constexpr int mod_pos(int x, int w) { return ((x % w) + w) % w; }
__host__ __device__ constexpr double inv_factorial(int j) {
    double f = 1.0;
    for (int k = 2; k <= j; ++k) f *= k;
    return 1.0 / f;
}
// (-i)^j = sign_re(j) on the real part / sign_im(j) on the imaginary part
// after the swap of roles: re_j = s_{j-1}, im_j = -re_{j-1}, re_0 = im_0 = +1.
__host__ __device__ constexpr double sign_re(int j) {
    double re = 1.0, im = 1.0;
    for (int k = 1; k <= j; ++k) { const double r = im, s = -re; re = r; im = s; }
    return re;
}
__host__ __device__ constexpr double sign_im(int j) {
    double re = 1.0, im = 1.0;
    for (int k = 1; k <= j; ++k) { const double r = im, s = -re; re = r; im = s; }
    return im;
}
__device__ __forceinline__ int wrap(int x, int n) { int r = x % n; return r < 0 ? r + n : r; }

template <typename T> __device__ __forceinline__ const T* jpar(const StepArgs& a);
template <> __device__ __forceinline__ const float* jpar<float>(const StepArgs& a) { return a.Jf; }
template <> __device__ __forceinline__ const double* jpar<double>(const StepArgs& a) { return a.Jd; }
template <typename T> __device__ __forceinline__ const T* epar(const StepArgs& a);
template <> __device__ __forceinline__ const float* epar<float>(const StepArgs& a) { return a.Ef; }
template <> __device__ __forceinline__ const double* epar<double>(const StepArgs& a) { return a.Ed; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Wave-uniform tables (row couplings) are read through the constant address
// space so that they land in scalar registers.
template <typename T> using UniformPtr = const __attribute__((address_space(4))) T*;

// A table entry read word by word through the constant address space (a
// struct copy cannot bind to that address space).
template <typename S>
__device__ __forceinline__ S load_uniform(const S* table, int index) {
    static_assert(sizeof(S) % 4 == 0, "word-sized entries");
    S v;
    const UniformPtr<int32_t> src = (UniformPtr<int32_t>)(table + index);
    int32_t* dst = reinterpret_cast<int32_t*>(&v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(S) / 4); ++k) dst[k] = src[k];
    return v;
}

// CHUNK: one pass of a chunked step (see StepArgs): the series continues
// from Psi_s with run-time coefficients, the partial sum comes from acc_in,
// and Psi_{s+NT} is stored for the next pass.
template <typename T, int NT, int P, bool KAHAN, bool TRI, bool CHUNK = false, bool VEC = false>
__device__ __forceinline__ void process_item(const StepArgs& a, int home, int lane) {
    using C = typename CplxOf<T>::type;
    constexpr int WA = window_rows(NT);
    // Rows fetched ahead: a whole window for complex64 (512-byte rows need
    // many loads in flight to cover the HBM latency), three for complex128
    // (1 KB rows, and the registers are taken by the wider windows) and for
    // chunked passes (which fetch two rows per row).
    constexpr int PF = (sizeof(T) == 4 && !CHUNK && P == 1) ? WA : 3;
    static_assert(WA % PF == 0, "the prefetch ring must tile the unrolled block");

    // The item and its realisation are wave-uniform: scalar loads, so every
    // pointer and row base derived from them stays in scalar registers.
    const ItemDev it = load_uniform(a.items, home);
    const RealDev rd = load_uniform(a.reals, it.real);
    const int N = rd.N;
    const int rows = rd.rows;
    const int nrows = it.nrows;
    const bool periodic = (rd.flags & RF_PERIODIC) != 0;
    const bool nearest = (rd.flags & RF_NEAREST) != 0;
    // two fermions in the triangle: the diagonal stays 0 and no coupling
    // doubles (the mirrored neighbours across it are the diagonal itself)
    const bool fermi = TRI && (rd.flags & RF_FERMION) != 0;
    // J and eps below are scaled by dt (host tables).
    const T* __restrict__ Jc = jpar<T>(a) + rd.param_off;
    const T* __restrict__ Ec = epar<T>(a) + rd.param_off;
    const UniformPtr<T> Jr = (UniformPtr<T>)(jpar<T>(a) + rd.row_param_off);
    const UniformPtr<T> Er = (UniformPtr<T>)(epar<T>(a) + rd.row_param_off);
    const C* __restrict__ in = reinterpret_cast<const C*>(a.psi_in) + rd.state_off;
    C* __restrict__ out = reinterpret_cast<C*>(a.psi_out) + rd.state_off;
    const T sc = (!CHUNK || a.first) ? static_cast<T>(((UniformPtr<double>)a.scale)[it.real]) : T(1);
    const T Udt = static_cast<T>(rd.U * a.dt);
    const C* __restrict__ acc_in = reinterpret_cast<const C*>(CHUNK ? a.acc_in : a.psi_in) + rd.state_off;
    C* __restrict__ seed_out = reinterpret_cast<C*>(CHUNK ? a.seed_out : a.psi_out) + rd.state_off;
    const bool keep_seed = CHUNK && a.seed_out != nullptr;
    const bool final_pass = !CHUNK || a.last;

    // Columns held by this lane.  Lanes outside [0, N) of an open chain hold
    // zeros with zero couplings, so they stay zero at every level.
    int col[P], colw[P];
    bool inb[P], outv[P];
    T jl[P], jr[P], ec[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int c = it.w0 + lane * P + p;
        col[p] = c;
        const int cw = periodic ? wrap(c, N) : c;
        colw[p] = cw;
        inb[p] = periodic || (c >= 0 && c < N);
        outv[p] = (c >= it.lo && c < it.hi);
        const int cs = inb[p] ? cw : 0;   // clamped: no access outside [0, N)
        jl[p] = inb[p] ? Jc[wrap(cs - 1, N)] : T(0);
        jr[p] = inb[p] ? Jc[cs] : T(0);
        ec[p] = inb[p] ? Ec[cs] : T(0);
    }

    // Row of the grid (wrapped on a ring) -> its stored amplitudes.  The
    // loads are unconditional (lanes without a stored amplitude read the
    // row's first one) so that the prefetch never waits; the mask is applied
    // when the row is consumed.  The row base is wave-uniform and each lane
    // adds a fixed byte offset, so a load needs no per-row vector arithmetic
    // (full grid; the triangle's mask moves with the row).
    uint32_t loff[P];
    T lmul[P];                      // load scale, 0 on lanes without an amplitude
#pragma unroll
    for (int p = 0; p < P; ++p) {
        loff[p] = inb[p] ? (uint32_t)colw[p] * (uint32_t)sizeof(C) : 0u;
        lmul[p] = inb[p] ? sc : T(0);
    }
    // Full grid, one pass per step (BUF): rows are read and written with
    // buffer instructions on a per-row resource (base and length of the row
    // in scalar registers) and a fixed per-lane offset.  Lanes off the
    // chain, or without an output column, use an offset past the row, which
    // reads zero and drops the store; a row past the sweep is fetched with
    // length 0 and reads zero.  So a row needs no per-lane address
    // arithmetic and no masking when it enters.
    // VEC (complex64, two columns per lane): every lane's two columns are
    // either both on the chain and adjacent in memory or both off it, and
    // the band's output columns start and end on even columns (the host
    // groups such items: even chain length, even window start and bounds).
    // A row is then one 16-byte access per lane, so that every access
    // instruction covers whole cache lines.
    constexpr bool BUF = !TRI && !CHUNK;
    static_assert(!VEC || (P == 2 && sizeof(T) == 4 && BUF), "paired access: complex64, P = 2");
    constexpr uint32_t kPastRow = 0x80000000u;
    uint32_t voff_in[P], voff_out[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        voff_in[p] = inb[p] ? loff[p] : kPastRow;
        voff_out[p] = outv[p] ? loff[p] : kPastRow;
    }
    const uint32_t row_bytes = (uint32_t)N * (uint32_t)sizeof(C);
    // the renormalisation scale of the input (1 unless renormalising)
    const bool scaled = sc != T(1);
    auto load_from = [&](const C* __restrict__ src, int qm, bool live_row, C (&dst)[P]) {
        const int base = TRI ? qm * N - (qm * (qm + 1)) / 2 : qm * N;
        const char* row = reinterpret_cast<const char*>(src + base);
        if constexpr (BUF) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<char*>(row), 0, live_row ? (int)row_bytes : 0, kBufferWord3);
            if constexpr (VEC) {
                const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff_in[0], 0, 0);
                dst[0].x = __uint_as_float(v.x);
                dst[0].y = __uint_as_float(v.y);
                dst[P - 1].x = __uint_as_float(v.z);
                dst[P - 1].y = __uint_as_float(v.w);
            } else {
#pragma unroll
                for (int p = 0; p < P; ++p) dst[p] = buffer_load_cplx<C>(rs, voff_in[p]);
            }
            return;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            uint32_t off = loff[p];
            if (TRI && col[p] < qm) off = 0u;
            dst[p] = *reinterpret_cast<const C*>(row + off);
        }
    };
    auto load_row = [&](int qm, bool live_row, C (&dst)[P]) { load_from(in, qm, live_row, dst); };

    T fr[NT][3][P], fi[NT][3][P];   // Psi_j rows, j < NT
    T ar[WA][P], ai[WA][P];         // partial sums of the rows in flight
    T cr[WA][P], ci[WA][P];         // sum of the terms j >= 1 of the rows in flight (KAHAN)
    T dg[WA][P];                    // dt * diagonal of H on the rows in flight
    T ju[WA];                       // dt * bond above each row in flight (uniform)
    C pre[PF][P];                   // rows being fetched
    C prea[CHUNK ? PF : 1][P];      // chunked pass: their partial sums
    T pj[3], pe[3];                 // bond above and energy of the next rows (uniform)
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int p = 0; p < P; ++p) { fr[j][s][p] = T(0); fi[j][s][p] = T(0); }
#pragma unroll
    for (int w = 0; w < WA; ++w) {
        ju[w] = T(0);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            ar[w][p] = ai[w][p] = cr[w][p] = ci[w][p] = dg[w][p] = T(0);
        }
    }
    // Grid rows are tracked incrementally: qm_in is the row entering at the
    // current iteration, qm_pf the one fetched PF iterations ahead and qm_pp
    // the one whose couplings are read three iterations ahead.  (Holding the
    // fetch on the sweep's last row instead of running past it measured the
    // same.)
    auto next_row = [&](int x) { return (x + 1 == rows) ? 0 : x + 1; };
    auto fetch_params = [&](int qm, int s) {
        pj[s] = Jr[qm == 0 ? rows - 1 : qm - 1];   // the padded last bond is 0 on an open chain
        pe[s] = Er[qm];
    };
    int qm_in = periodic ? wrap(it.row0, rows) : it.row0;
    int qm_pf = qm_in, qm_pp = qm_in;
    auto advance_pf = [&]() { qm_pf = next_row(qm_pf); };
#pragma unroll
    for (int s = 0; s < PF; ++s) {   // rows past the sweep are fetched and ignored
        load_row(qm_pf, s < nrows, pre[s]);
        if constexpr (CHUNK) load_from(acc_in, qm_pf, true, prea[s]);
        advance_pf();
        // Keep the prologue loads in slot order: the sweep consumes slot 0
        // first, and the wait it needs is then for the oldest load only.
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        fetch_params(qm_pp, s);
        qm_pp = next_row(qm_pp);
    }

    // Norm weights of this lane's outputs (full grid: 1 on the band's output
    // columns; triangle: 2 off the diagonal, set per row).
    double wcol[P];
#pragma unroll
    for (int p = 0; p < P; ++p) wcol[p] = outv[p] ? 1.0 : 0.0;

    double nrm = 0.0, tail = 0.0;   // triangle: weighted per row
    // Full grid: per column, weighted at the end.  The squared norm sums
    // exact FP64 squares; the last term's squared norm only scales the
    // remainder bound, so it is summed in the state's precision (relative
    // error below 1e-4 for complex64 over any sweep) and widened at the end.
    double nrmp[P];
    T tailp[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        nrmp[p] = 0.0;
        tailp[p] = T(0);
    }
    // The sweep runs nrows + NT iterations, rounded up to whole unrolled
    // blocks: the extra iterations see zero rows and store nothing, and the
    // block body has no early exit (which keeps the prefetch waits exact).
    const int total = nrows + NT;

    // One unrolled block of WA sweep steps.  ND: every level's rows have a
    // zero diagonal on every lane, so the stencil skips the diagonal product.
    auto block = [&](auto nodiag, int i0) {
        constexpr bool ND = decltype(nodiag)::value;
#pragma unroll
        for (int u = 0; u < WA; ++u) {
            const int i = i0 + u;
            {
                // ---- level 0: row i enters (zero beyond the sweep).  The
                // bond above a row beyond the sweep is 0, so nothing flows
                // back from there.
                {
                    const int s = u % 3;
                    const int sp = u % PF;
                    const bool live = i < nrows;
                    const int qm = qm_in;
                    C v[P], va[P];
                    T mul[P];
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        v[p] = pre[sp][p];
                        va[p] = CHUNK ? prea[sp][p] : v[p];
                        // zero past the sweep and off the stored lanes (incl. the triangle's lower part)
                        mul[p] = BUF ? T(1) : ((live && (!TRI || col[p] >= qm)) ? lmul[p] : T(0));
                    }
                    const T er = pe[s];
                    ju[u] = live ? pj[s] : T(0);
                    // consume the slot before it is refilled (no copy of the old row)
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        T re, im;
                        if constexpr (BUF) {
                            // zero off the chain and past the sweep already
                            re = v[p].x;
                            im = v[p].y;
                            if (scaled) {
                                re *= sc;
                                im *= sc;
                            }
                        } else {
                            re = v[p].x * mul[p];
                            im = v[p].y * mul[p];
                        }
                        fr[0][s][p] = re;
                        fi[0][s][p] = im;
                        ar[u][p] = CHUNK ? va[p].x * mul[p] : re;
                        ai[u][p] = CHUNK ? va[p].y * mul[p] : im;
                    }
                    load_row(qm_pf, i + PF < nrows, pre[sp]);
                    if constexpr (CHUNK) load_from(acc_in, qm_pf, true, prea[sp]);
                    fetch_params(qm_pp, s);
                    // The columns that interact with row qm (wave-uniform): qm itself
                    // (on site), or qm - 1 and qm + 1 (nearest, wrapped on a ring;
                    // off the chain they match no stored column).  -2^30: none.
                    int t1 = -(1 << 30), t2 = -(1 << 30);
                    if (rows > 1) {
                        if (nearest) {
                            t1 = qm - 1;
                            t2 = qm + 1;
                            if (periodic) {
                                t1 = t1 < 0 ? t1 + N : t1;
                                t2 = t2 >= N ? t2 - N : t2;
                            }
                        } else {
                            t1 = qm;
                        }
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        T d0 = er + ec[p];
                        if (colw[p] == t1 || colw[p] == t2) d0 += Udt;
                        dg[u][p] = d0;
                    }
                    qm_in = next_row(qm_in);
                    advance_pf();
                    qm_pp = next_row(qm_pp);
                }
                // ---- levels 1..NT: Psi_j on row i - j.
#pragma unroll
                for (int j = 1; j <= NT; ++j) {
                    const int su = mod_pos(u - j - 1, 3);
                    const int sm = mod_pos(u - j, 3);
                    const int sd = mod_pos(u - j + 1, 3);
                    const int w = mod_pos(u - j, WA);
                    const int w1 = mod_pos(u - j + 1, WA);
                    const T Ju = ju[w];
                    const T Jd = ju[w1];
                    // Psi_j = sr_j A_j + i si_j B_j with A_j = H B_{j-1}, B_j = H A_{j-1}:
                    // the factor -i only swaps the two parts and moves signs, which are
                    // compile-time and folded into the accumulation coefficients.
                    const T f_j = CHUNK ? static_cast<T>(a.coef[j - 1]) : static_cast<T>(inv_factorial(j));
                    const T cr_j = static_cast<T>(sign_re(j)) * f_j;
                    const T ci_j = static_cast<T>(sign_im(j)) * f_j;
                    // Triangle: the band's rows at and below its first column hold the
                    // diagonal; there the couplings up and right double and the
                    // lower triangle is held at zero.
                    const int qa = it.row0 + (i - j);
                    const bool zone = TRI && qa >= it.w0;
                    T hrv[P], hiv[P];
                    if constexpr (sizeof(T) == 4 && !TRI) {
                        if constexpr (ND) {
                            if constexpr (P == 1)
                                stencil_c64_p1_nd(hrv[0], hiv[0], fr[j - 1][sm][0], fi[j - 1][sm][0],
                                                  fr[j - 1][su][0], fi[j - 1][su][0], fr[j - 1][sd][0],
                                                  fi[j - 1][sd][0], Ju, Jd, jl[0], jr[0]);
                            else
                                stencil_c64_p2_nd(hrv, hiv, fr[j - 1][sm], fi[j - 1][sm], fr[j - 1][su],
                                                  fi[j - 1][su], fr[j - 1][sd], fi[j - 1][sd], Ju, Jd, jl, jr);
                        } else {
                            if constexpr (P == 1)
                                stencil_c64_p1(hrv[0], hiv[0], dg[w][0], fr[j - 1][sm][0], fi[j - 1][sm][0],
                                               fr[j - 1][su][0], fi[j - 1][su][0], fr[j - 1][sd][0],
                                               fi[j - 1][sd][0], Ju, Jd, jl[0], jr[0]);
                            else
                                stencil_c64_p2(hrv, hiv, dg[w], fr[j - 1][sm], fi[j - 1][sm], fr[j - 1][su],
                                               fi[j - 1][su], fr[j - 1][sd], fi[j - 1][sd], Ju, Jd, jl, jr);
                        }
                    } else {
                        T lr[P], li[P], rr[P], ri[P];
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            if (p > 0) { lr[p] = fr[j - 1][sm][p - 1]; li[p] = fi[j - 1][sm][p - 1]; }
                            if (p < P - 1) { rr[p] = fr[j - 1][sm][p + 1]; ri[p] = fi[j - 1][sm][p + 1]; }
                        }
                        lr[0] = from_left(fr[j - 1][sm][P - 1]);
                        li[0] = from_left(fi[j - 1][sm][P - 1]);
                        rr[P - 1] = from_right(fr[j - 1][sm][0]);
                        ri[P - 1] = from_right(fi[j - 1][sm][0]);
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            T cu = Ju, crt = jr[p];
                            if (TRI && zone && col[p] == qa && !fermi) { cu = Ju + Ju; crt = crt + crt; }
                            const T mr = fr[j - 1][sm][p], mi = fi[j - 1][sm][p];
                            T hr, hi;
                            if constexpr (ND) {
                                hr = cu * fr[j - 1][su][p];
                                hi = cu * fi[j - 1][su][p];
                            } else {
                                hr = dg[w][p] * mr;
                                hi = dg[w][p] * mi;
                                hr += cu * fr[j - 1][su][p];
                                hi += cu * fi[j - 1][su][p];
                            }
                            hr += Jd * fr[j - 1][sd][p];
                            hi += Jd * fi[j - 1][sd][p];
                            hr += jl[p] * lr[p];
                            hi += jl[p] * li[p];
                            hr += crt * rr[p];
                            hi += crt * ri[p];
                            hrv[p] = hr;
                            hiv[p] = hi;
                        }
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const bool low = TRI && zone && (col[p] < qa || (fermi && col[p] == qa));
                        const T hr = hrv[p], hi = hiv[p];
                        // A_j = H B_{j-1} (from the imaginary-role array), B_j = H A_{j-1}
                        T pr_ = hi;
                        T pi_ = hr;
                        if (TRI && low) { pr_ = T(0); pi_ = T(0); }
                        if (j < NT) { fr[j % NT][sm][p] = pr_; fi[j % NT][sm][p] = pi_; }
                        if (KAHAN && j == 1) {
                            // The terms are summed apart from psi (they are
                            // smaller than psi by x = dt ||H|| or more) and
                            // added to it once, when the row is complete.
                            cr[w][p] = cr_j * pr_;   // fused step: cr_1, ci_1 = +-1
                            ci[w][p] = ci_j * pi_;
                        } else if (KAHAN) {
                            cr[w][p] = fma_t(cr_j, pr_, cr[w][p]);
                            ci[w][p] = fma_t(ci_j, pi_, ci[w][p]);
                        } else {
                            ar[w][p] += cr_j * pr_;
                            ai[w][p] += ci_j * pi_;
                        }
                        const bool tail_here = CHUNK ? (final_pass && j == a.tail_level) : (j == NT);
                        if (tail_here) {
                            const int q = i - j;
                            if (q >= 0 && qa >= it.out_lo && qa < it.out_hi) {
                                const double dr = pr_, di = pi_;
                                if (TRI) {
                                    const double wgt =
                                        (col[p] > qa) ? 2.0 * wcol[p] : (col[p] == qa ? wcol[p] : 0.0);
                                    tail = __builtin_fma(wgt, __builtin_fma(di, di, dr * dr), tail);
                                } else {   // column weight applied once at the end
                                    tailp[p] = fma_t(pr_, pr_, tailp[p]);
                                    tailp[p] = fma_t(pi_, pi_, tailp[p]);
                                }
                            }
                        }
                        if (CHUNK && j == NT && keep_seed) {
                            // Psi_{s+NT} of row i - NT, with its true signs, for the next pass
                            const int q = i - NT;
                            if (q >= 0 && qa >= it.out_lo && qa < it.out_hi && outv[p] && (!TRI || col[p] >= qa)) {
                                const int base = TRI ? qa * N - (qa * (qa + 1)) / 2 : qa * N;
                                C sv;
                                sv.x = static_cast<T>(sign_re(NT)) * pr_;
                                sv.y = static_cast<T>(sign_im(NT)) * pi_;
                                *reinterpret_cast<C*>(reinterpret_cast<char*>(seed_out + base) + loff[p]) = sv;
                            }
                        }
                    }
                }
                // ---- row i - NT is complete.
                {
                    const int q = i - NT;
                    const int w = mod_pos(u - NT, WA);
                    const int qa = it.row0 + q;
                    if (q >= 0 && qa >= it.out_lo && qa < it.out_hi) {
                        const int base = TRI ? qa * N - (qa * (qa + 1)) / 2 : qa * N;
                        C vo[P];
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            vo[p].x = KAHAN ? ar[w][p] + cr[w][p] : ar[w][p];
                            vo[p].y = KAHAN ? ai[w][p] + ci[w][p] : ai[w][p];
                        }
                        if constexpr (BUF) {
                            const __amdgpu_buffer_rsrc_t rs =
                                __builtin_amdgcn_make_buffer_rsrc(out + base, 0, (int)row_bytes, kBufferWord3);
                            if constexpr (VEC) {
                                u32x4 v4;
                                v4.x = __float_as_uint(vo[0].x);
                                v4.y = __float_as_uint(vo[0].y);
                                v4.z = __float_as_uint(vo[P - 1].x);
                                v4.w = __float_as_uint(vo[P - 1].y);
                                __builtin_amdgcn_raw_buffer_store_b128(v4, rs, (int)voff_out[0], 0, kStorePolicy);
                            } else {
#pragma unroll
                                for (int p = 0; p < P; ++p) buffer_store_cplx(vo[p], rs, voff_out[p]);
                            }
                        }
#pragma unroll
                        for (int p = 0; p < P; ++p) {
                            const C v = vo[p];
                            if (!BUF && outv[p] && (!TRI || col[p] >= qa))
                                *reinterpret_cast<C*>(reinterpret_cast<char*>(out + base) + loff[p]) = v;
                            if (final_pass) {
                                const double dr = v.x, di = v.y;
                                if (TRI) {
                                    const double wgt =
                                        (col[p] > qa) ? 2.0 * wcol[p] : (col[p] == qa ? wcol[p] : 0.0);
                                    nrm = __builtin_fma(wgt, __builtin_fma(di, di, dr * dr), nrm);
                                } else {
                                    nrmp[p] = __builtin_fma(dr, dr, nrmp[p]);
                                    nrmp[p] = __builtin_fma(di, di, nrmp[p]);
                                }
                            }
                        }
                    }
                }
            }
        }
    };
    // Without on-site energies the diagonal of H is the interaction alone,
    // nonzero only on the rows whose interacting columns (the row itself on
    // site, its neighbours for nearest-neighbour pairs) fall in the band's
    // window: the levels of other rows skip the diagonal product.  Steps
    // [d0, d1) (whole blocks) hold a level on such a row; the diagonal of
    // every row is still formed at level 0, so the slots stay exact.
    int d0 = 0, d1 = total;
    if constexpr (!TRI && !CHUNK) {
        if ((rd.flags & RF_NO_EPS) && !periodic && rows > 1) {
            const int reach = nearest ? 1 : 0;
            const int zlo = max(0, it.w0 - reach - it.row0);
            const int zhi = min(nrows, it.w0 + 64 * P + reach - it.row0);
            if (Udt == T(0) || zlo >= zhi) {
                d0 = d1 = 0;
            } else {
                d0 = ((zlo + 1) / WA) * WA;
                d1 = ((zhi + NT + WA - 1) / WA) * WA;
            }
        }
        int i0 = 0;
        for (; i0 < d0 && i0 < total; i0 += WA) block(std::true_type{}, i0);
        for (; i0 < d1 && i0 < total; i0 += WA) block(std::false_type{}, i0);
        for (; i0 < total; i0 += WA) block(std::true_type{}, i0);
    } else {
        for (int i0 = 0; i0 < total; i0 += WA) block(std::false_type{}, i0);
    }
    if (!TRI) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            nrm = __builtin_fma(wcol[p], nrmp[p], nrm);
            tail = __builtin_fma(wcol[p], (double)tailp[p], tail);
        }
    }
    nrm = wave_sum(nrm);
    tail = wave_sum(tail);
    if (lane == 0 && final_pass) {
        const double f = CHUNK ? a.tail_coef : inv_factorial(NT);
        a.norm_part[home] = nrm;
        a.tail_part[home] = tail * f * f;
    }
}

// One kernel serves both launch forms.  Items are taken in groups of one
// item per wave of the block.  Regular: block b takes group b of the
// processing order and the hardware hands out the blocks.  Persistent (a
// grid of resident blocks): the processing order is split into kClaimLists
// lists, list x holding work for the blocks on XCD x (b mod kClaimLists);
// the adjacent bands of a realisation sit next to each other in one list,
// so that their overlapping columns are read through one L2 at about the
// same time.  A block claims the next group of its list from that list's
// counter (zeroed by the host before the launch); when its list is used up
// it moves on to the next list, and it leaves after kClaimLists claims in a
// row past the ends of lists (counters only grow, so every list is then
// used up).  Lane 0 of wave 0 alone adds 1 to the counter (one claim per
// add, whatever the compiler does with atomics of several lanes) and passes
// the old value to the block through LDS (two slots used alternately, so a
// slot is rewritten only after every wave has passed the next barrier);
// every wave reads it back with readfirstlane, so the loop's branches are
// uniform over the block and every wave meets every barrier.
// Static assignments of items to waves (round-robin,
// longest-processing-time) ran 20 % slower: the resident waves do not all
// advance at the same rate, and only claiming at run time follows that.
// Two columns per lane in complex64 up to 7 terms sit at the 256-VGPR line
// (two waves per SIMD); ask the compiler to stay under it.
template <typename T, int NT, int P, bool CHUNK>
constexpr int min_blocks_per_cu() {
    return (P == 2 && sizeof(T) == 4 && NT <= 7 && !CHUNK) ? 2 : 1;
}

// TWO: the launch holds items of two orders, NT and NT - 1 (mixed in one
// largest-first list, so that the instruction-heavier and the lighter items
// share the device instead of running as two phases); each item runs at
// its realisation's order.
template <typename T, int NT, int P, bool KAHAN, bool TRI, bool CHUNK = false, bool VEC = false, bool TWO = false>
__global__ void __launch_bounds__(256, (min_blocks_per_cu<T, NT, P, CHUNK>())) step2d_kernel(StepArgs a) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ int next_group[2];
    // One loop for both forms, so the item code is inlined once and both
    // forms run the same instructions: a regular launch runs group
    // blockIdx.x of the whole order once.
    int x = (int)(blockIdx.x % kClaimLists);
    int end = a.n_items;   // end of the current list (regular: of the order)
    int first = (int)blockIdx.x * wpb;
    int it = 0;
    if (a.persistent) first = a.n_items;   // no group yet: claim below
    // One loop for both forms, so the item code is inlined once and both
    // forms run the same instructions: a regular launch runs group
    // blockIdx.x of the whole order and leaves.
    for (bool started = !a.persistent;;) {
        if (started) {
            const int k = first + wv;
            if (k < end) {
                const int home = ((UniformPtr<int32_t>)a.item_order)[k];
                if constexpr (TWO) {
                    static_assert(NT >= 2 && !CHUNK, "two orders: NT and NT - 1");
                    const int real = ((UniformPtr<int32_t>)(a.items + home))[0];
                    if (load_uniform(a.reals, real).order == NT)
                        process_item<T, NT, P, KAHAN, TRI, CHUNK, VEC>(a, home, lane);
                    else
                        process_item<T, (TWO ? NT - 1 : NT), P, KAHAN, TRI, CHUNK, VEC>(a, home, lane);
                } else {
                    process_item<T, NT, P, KAHAN, TRI, CHUNK, VEC>(a, home, lane);
                }
            }
            if (!a.persistent) break;
        }
        started = true;
        // Claim the next group of list x, or of the lists after it.
        // (x, the bounds and the claim are block-uniform; readfirstlane
        // keeps them, and everything derived from them, in scalar registers)
        int misses = 0;
        for (; misses < kClaimLists; ++misses, ++it) {
            x = __builtin_amdgcn_readfirstlane(x);
            if (wv == 0 && lane == 0) next_group[it & 1] = atomicAdd(a.claim + x, 1);
            __syncthreads();
            const int lo = __builtin_amdgcn_readfirstlane(((UniformPtr<int32_t>)a.list_off)[x]);
            end = __builtin_amdgcn_readfirstlane(((UniformPtr<int32_t>)a.list_off)[x + 1]);
            first = lo + __builtin_amdgcn_readfirstlane(next_group[it & 1]) * wpb;
            if (first < end) break;
            x = (x + 1 == kClaimLists) ? 0 : x + 1;   // list x is used up
        }
        if (misses == kClaimLists) break;
        ++it;
    }
}

}  // namespace step2d_detail

using StepKernelFn = void (*)(StepArgs);

}  // namespace ctqw

// Table of compiled pipeline depths for one (type, columns per lane,
// accumulation, layout) combination; each translation unit instantiates one.
#define CTQW_STEP_CASE(T, NT, P, K, TRI) \
    case NT: return &::ctqw::step2d_detail::step2d_kernel<T, NT, P, K, TRI>;
#define CTQW_STEP_CASE_VEC(T, NT, K) \
    case NT: return &::ctqw::step2d_detail::step2d_kernel<T, NT, 2, K, false, false, true>;
#define CTQW_STEP_CASE_TWO(T, NT, P, K, VEC) \
    case NT: return &::ctqw::step2d_detail::step2d_kernel<T, NT, P, K, false, false, VEC, true>;
