// Three particles on a chain: K Taylor terms chained per pass over the state.
//
// The walk of m = 3 distinguishable particles lives on the N^3 grid
// psi[x1][x2][x3] (x3 fastest).  A step of Alg. 3 (Eqs. 6-7) needs n terms
// Phi^(j) = -(i dt / j) H Phi^(j-1); this kernel computes K of them per pass,
// so a step is ceil(n / K) passes.  Pass q continues the series from
// X = Psi_s = (-i dt H)^s psi (s = qK; X = psi on the first pass): it forms
// Y_j = (dt H)^j X for j = 1..K, adds sum_j (-i)^j Y_j / (s + j)! to the
// partial sum, and hands Psi_{s+K} = (-i)^K Y_K to the next pass.  H is
// applied matrix-free (Eq. 1 with the Kronecker-sum structure):
//   (H y)(x) = sum_a J[x_a - 1] y(x - e_a) + J[x_a] y(x + e_a)
//            + (eps[x1] + eps[x2] + eps[x3] + V(x)) y(x),
// V = U * #{a < b : chain distance |x_a - x_b| == 1} (nearest neighbours) or
// U * #{a < b : x_a == x_b} (on site); the tables hold dt-scaled J and eps.
//
// Work item: a tile of the (x2, x3) plane -- 64 x3 columns (one per lane)
// by W*S x2 rows (S consecutive rows per wave, W waves per block) -- swept
// over every x1 plane.  A pipeline of K levels runs down the planes: at
// sweep step i the plane i enters level 0, level j computes plane i - j from
// level j-1's planes i-j-1, i-j, i-j+1 (all in registers), and plane i - K
// is complete and stored.  Within a plane, x3 neighbours are the adjacent
// lanes (DPP row shifts) and x2 neighbours the wave's own rows; the rows
// just above and below a wave's strip belong to the neighbouring waves,
// which publish their first and last rows of every level in LDS once per
// sweep step (double-buffered: one barrier per step).  The tile overlaps
// its neighbours by K columns and K rows (the halo), recomputed by both;
// x1 needs no halo on an open chain (the sweep runs the whole axis).
//
// HBM traffic per amplitude and pass: read X (and the partial sum after the
// first pass), write the partial sum (and Psi_{s+K} before the last pass):
// with n = 2K terms, 24 + 24 = 48 bytes (complex64) per step instead of
// one read and one write per term.  The terms of a pass are summed apart
// from the partial sum and added to it once, so the new state takes one
// rounding per pass.
#include "step3c.hpp"

namespace ctqw {
namespace step3c_detail {

template <typename T> struct Cplx3c;
template <> struct Cplx3c<float> { using type = float2; };
template <> struct Cplx3c<double> { using type = double2; };

// Lane l receives lane l-1 (lane 0 receives 0) / lane l+1 (lane 63: 0).
__device__ __forceinline__ float lane_from_left(float x) {
    return __builtin_amdgcn_update_dpp(0.0f, x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ double lane_from_left(double x) {
    return __builtin_amdgcn_update_dpp(0.0, x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ float lane_from_right(float x) {
    return __builtin_amdgcn_update_dpp(0.0f, x, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ double lane_from_right(double x) {
    return __builtin_amdgcn_update_dpp(0.0, x, 0x130, 0xF, 0xF, true);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufferWord3 = 0x00020000;
constexpr int kStoreNT = 2;   // stores are read again only by the next pass
constexpr uint32_t kPastRow = 0x80000000u;

// Loads and stores of one amplitude per lane through a buffer resource over
// one plane, row and column in the per-lane offset and a zero scalar offset.
// An offset at or past the resource's length reads 0 and drops the store.
// (A 16-byte store reads its data registers after it issues: a VALU write
// of them must wait one cycle.  The compiler inserts that wait only for
// stores whose scalar offset is not a register; with a register there the
// store was seen to write the following instruction's results in some
// lanes.  A zero scalar offset keeps the wait.)
__device__ __forceinline__ float2 load_c(__amdgpu_buffer_rsrc_t rs, uint32_t off, float2*) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
__device__ __forceinline__ double2 load_c(__amdgpu_buffer_rsrc_t rs, uint32_t off, double2*) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    return make_double2(__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z));
}
__device__ __forceinline__ void store_c(float re, float im, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x2 v;
    v.x = __float_as_uint(re);
    v.y = __float_as_uint(im);
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, (int)off, 0, kStoreNT);
}
__device__ __forceinline__ void store_c(double re, double im, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x4 v;
    v.x = (unsigned)__double2loint(re);
    v.y = (unsigned)__double2hiint(re);
    v.z = (unsigned)__double2loint(im);
    v.w = (unsigned)__double2hiint(im);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, kStoreNT);
}

template <typename T> using UPtr = const __attribute__((address_space(4))) T*;

template <typename S>
__device__ __forceinline__ S load_uniform3(const S* table, int index) {
    static_assert(sizeof(S) % 4 == 0, "word-sized entries");
    S v;
    const UPtr<int32_t> src = (UPtr<int32_t>)(table + index);
    int32_t* dst = reinterpret_cast<int32_t*>(&v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(S) / 4); ++k) dst[k] = src[k];
    return v;
}

__device__ __forceinline__ int wrap3(int x, int n) { int r = x % n; return r < 0 ? r + n : r; }
__host__ __device__ constexpr int m3(int x) { return ((x % 3) + 3) % 3; }
// (-i)^j = sr + i si with (sr, si) applied after the swap of roles: for odd
// j the real part of (-i)^j y is si_j * Im y, the imaginary part sr_j * Re y.
__host__ __device__ constexpr float rot_re(int j) { return (j % 4 == 0 || j % 4 == 1) ? 1.0f : -1.0f; }
__host__ __device__ constexpr float rot_im(int j) { return (j % 4 == 0 || j % 4 == 3) ? 1.0f : -1.0f; }

// Chain distance |a - b| (the shorter way round on a ring) == want, without branches.
__device__ __forceinline__ bool related_u(int a, int b, int N, bool periodic, int want) {
    const int d = a > b ? a - b : b - a;
    const int e = N - d;
    return ((periodic && e < d) ? e : d) == want;
}

// The complex64 stencil of one amplitude and level, h = (dt H y)(x):
//   h = d m + Ju u + Jd v + Ja a + Jb b + jl m(lane - 1) + jr m(lane + 1)
// (m: this amplitude; u, v: the planes above and below; a, b: the rows
// above and below; Ju, Jd, Ja, Jb wave-uniform bonds; jl, jr the lane's
// x3 bonds), accumulated in this order for the real and imaginary parts.
// The x3 neighbours are read from the adjacent lanes by the FMA itself
// (DPP wave_shr / wave_shl, bound_ctrl: lanes 0 and 63 read 0).  A DPP read
// of a VGPR must follow the VALU write of that register by two wait
// states: the DPP instructions come after ten VALU instructions of the
// block and read inputs of the block.
__device__ __forceinline__ void stencil3_c64(float& hr, float& hi, float d, float mr, float mi, float ur, float ui,
                                             float vr, float vi, float ar, float ai, float br, float bi, float Ju,
                                             float Jd, float Ja, float Jb, float jl, float jr) {
    asm("v_mul_f32 %0, %2, %3\n\t"
        "v_mul_f32 %1, %2, %4\n\t"
        "v_fmac_f32 %0, %13, %5\n\t"
        "v_fmac_f32 %1, %13, %6\n\t"
        "v_fmac_f32 %0, %14, %7\n\t"
        "v_fmac_f32 %1, %14, %8\n\t"
        "v_fmac_f32 %0, %15, %9\n\t"
        "v_fmac_f32 %1, %15, %10\n\t"
        "v_fmac_f32 %0, %16, %11\n\t"
        "v_fmac_f32 %1, %16, %12\n\t"
        "v_fmac_f32_dpp %0, %3, %17 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %4, %17 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %0, %3, %18 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
        "v_fmac_f32_dpp %1, %4, %18 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=&v"(hr), "=&v"(hi)
        : "v"(d), "v"(mr), "v"(mi), "v"(ur), "v"(ui), "v"(vr), "v"(vi), "v"(ar), "v"(ai), "v"(br), "v"(bi),
          "s"(Ju), "s"(Jd), "s"(Ja), "s"(Jb), "v"(jl), "v"(jr));
}

__device__ __forceinline__ float fma3(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma3(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ double wave_sum3(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// FIRST: X = psi times the realisation's load scale, and the partial sum
// before the pass is X itself; LAST: the pass writes the new state, the
// FP64 squared norm of it and of the order's last term (the kernel's last
// level), and no Psi_{s+K}.  PROD (step3c.hpp): the pass writes
// X + sum_j c_j Y_j with complex c_j and no Psi_{s+K}; the first pass of a
// step forms the squared norm of its last level, which bounds the last term.
template <typename T, int KT, int S, int W, bool FIRST, bool LAST, bool PROD>
__global__ void __launch_bounds__(64 * W, 1) step3c_kernel(Step3cArgs a, Step3cProd pp) {
    using C = typename Cplx3c<T>::type;
    static_assert(KT >= 1 && KT <= 3, "windows are indexed modulo 3");
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Neighbour-row exchange: [buffer][level][wave slot][first/last row][lane];
    // wave w publishes in slot w + 1, slots 0 and W + 1 stay zero.
    __shared__ C edge[2][KT][W + 2][2][64];

    // Blocks are dealt to the XCDs round-robin; consecutive items (adjacent
    // tiles of one realisation) are given to blocks of one XCD, so that the
    // halo rows and columns they share are read through one L2.
    const int per_xcd = (a.n_items + 7) / 8;
    const int home = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (home >= a.n_items) return;   // whole block, before any barrier

    for (int k = threadIdx.x; k < 2 * KT * (W + 2) * 2 * 64; k += 64 * W) {
        C z;
        z.x = T(0);
        z.y = T(0);
        (&edge[0][0][0][0][0])[k] = z;
    }

    const Item3Dev it = load_uniform3(a.items, home);
    const RealDev rd = load_uniform3(a.reals, it.real);
    const int N = rd.N;
    const bool periodic = (rd.flags & RF_PERIODIC) != 0;
    const int want = (rd.flags & RF_NEAREST) ? 1 : 0;
    const T* __restrict__ Jt = reinterpret_cast<const T*>(a.Jt) + rd.param_off;
    const T* __restrict__ Et = reinterpret_cast<const T*>(a.Et) + rd.param_off;
    const UPtr<T> Ju_t = (UPtr<T>)(reinterpret_cast<const T*>(a.Jt) + rd.param_off);
    const UPtr<T> Eu_t = (UPtr<T>)(reinterpret_cast<const T*>(a.Et) + rd.param_off);
    const T Udt = static_cast<T>(rd.U * a.dt);
    const int64_t NN = (int64_t)N * N;
    const char* x_base = reinterpret_cast<const char*>(reinterpret_cast<const C*>(a.x_in) + rd.state_off);
    const char* b_base = reinterpret_cast<const char*>(reinterpret_cast<const C*>(a.base_in) + rd.state_off);
    char* s_base = reinterpret_cast<char*>(reinterpret_cast<C*>(a.sum_out) + rd.state_off);
    char* q_base = (LAST || PROD) ? s_base : reinterpret_cast<char*>(reinterpret_cast<C*>(a.seed_out) + rd.state_off);
    // which FP64 partials this pass forms: the new state's squared norm
    // (last pass) and the last term's (chained: last pass; product: first)
    constexpr bool DO_NORM = LAST;
    constexpr bool DO_TAIL = PROD ? FIRST : LAST;
    const T sc = FIRST ? static_cast<T>(((UPtr<double>)a.scale)[it.real]) : T(1);
    const int plane_bytes = (int)(NN * (int64_t)sizeof(C));

    // ---- this lane's x3 column
    const int z = it.z0 + lane;
    const int zw = periodic ? wrap3(z, N) : z;
    const bool zin = periodic || (z >= 0 && z < N);
    const bool zout = z >= it.zlo && z < it.zhi;
    const int zs = zin ? zw : 0;
    const T jl = zin ? Jt[wrap3(zs - 1, N)] : T(0);
    const T jr = zin ? Jt[zs] : T(0);
    const T e3 = zin ? Et[zs] : T(0);
    const uint32_t voff_in = zin ? (uint32_t)zw * (uint32_t)sizeof(C) : kPastRow;
    const uint32_t voff_out = (zin && zout) ? (uint32_t)zw * (uint32_t)sizeof(C) : kPastRow;
    // the planes x1 interacting with this lane's column (-1: none)
    const int zta = zin ? (periodic ? wrap3(zw - want, N) : zw - want) : -1;
    const int ztb = zin ? (periodic ? wrap3(zw + want, N) : zw + want) : -1;

    // ---- this wave's x2 rows (wave-uniform)
    bool yin[S];     // row on the chain: loads read it, else zero
    bool yout[S];    // output row: stores write it
    uint32_t voff_ld[S];   // the lane's row and column offset, past the plane off the chain
    uint32_t voff_st[S];   // the lane's row and column offset, past the plane off the output
    T jrow[S + 1];   // jrow[s]: dt * bond between rows s-1 and s of the strip
    T drow[S];       // per lane: dt * (eps[x2] + eps[x3] + interaction of (x2, x3))
    int ywr[S];
    int yta[S], ytb[S];   // planes x1 interacting with row s (-1: none)
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int y = it.y0 + wv * S + s;
        const int yw = periodic ? wrap3(y, N) : y;
        yin[s] = periodic || (y >= 0 && y < N);
        yout[s] = y >= it.ylo && y < it.yhi;
        ywr[s] = yin[s] ? yw : 0;
        const uint32_t soff = (uint32_t)ywr[s] * (uint32_t)N * (uint32_t)sizeof(C);   // the row in a plane
        voff_ld[s] = (yin[s] && voff_in != kPastRow) ? voff_in + soff : kPastRow;
        voff_st[s] = (yout[s] && voff_out != kPastRow) ? voff_out + soff : kPastRow;
        // the planes x1 whose interaction with this row counts (the chain
        // distance |x1 - x2| equals `want`; none off the chain)
        yta[s] = yin[s] ? (periodic ? wrap3(ywr[s] - want, N) : ywr[s] - want) : -1;
        ytb[s] = yin[s] ? (periodic ? wrap3(ywr[s] + want, N) : ywr[s] + want) : -1;
    }
#pragma unroll
    for (int s = 0; s <= S; ++s) {
        const int y = it.y0 + wv * S + s;
        const int ya = y - 1;
        const bool ok_hi = periodic || (y >= 0 && y < N);
        const bool ok_lo = periodic || (ya >= 0 && ya < N);
        const int b = (ok_hi && ok_lo) ? (periodic ? wrap3(ya, N) : ya) : 0;   // index in range either way
        const T jb = Ju_t[b];
        jrow[s] = (ok_hi && ok_lo) ? jb : T(0);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        T d = e3 + (yin[s] ? Eu_t[ywr[s]] : T(0));
        if (zin && yin[s] && related_u(ywr[s], zw, N, periodic, want)) d += Udt;
        drow[s] = d;
    }

    // ---- register windows (planes modulo 3)
    T yr[KT][3][S], yi[KT][3][S];   // Y_j, j < KT
    T tr[3][S], ti[3][S];           // sum of this pass's terms
    T br[3][S], bi[3][S];           // partial sum before this pass
    T dg[3][S];                     // dt * diagonal of H
    T jq[KT + 1];                   // dt * bond above planes i-KT .. i (uniform)
    C pre[3][S];                    // planes being fetched
#pragma unroll
    for (int k = 0; k <= KT; ++k) jq[k] = T(0);
#pragma unroll
    for (int w = 0; w < 3; ++w) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            tr[w][s] = ti[w][s] = br[w][s] = bi[w][s] = dg[w][s] = T(0);
#pragma unroll
            for (int j = 0; j < KT; ++j) yr[j][w][s] = yi[j][w][s] = T(0);
        }
    }

    const int nplanes = it.nplanes;
    const int plo = it.plane_lo - it.x0, phi = it.plane_hi - it.x0;   // output planes (sweep index)
    // Plane p of the sweep is x1 = x0 + p (wrapped on a ring); open chains
    // sweep exactly [0, N).  A plane is addressed through one buffer
    // resource (length 0 -- loads read zero, stores are dropped -- where `ok`
    // is false), the row as scalar offset and the column as lane offset.
    auto live = [&](int p) { return p >= 0 && p < nplanes; };
    auto plane_out = [&](int p) { return p >= plo && p < phi && p >= 0; };
    auto rsrc = [&](const char* base, int xw, bool ok) {
        const int64_t off = (int64_t)(ok ? xw : 0) * NN * (int64_t)sizeof(C);
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base + off), 0, ok ? plane_bytes : 0,
                                                 kBufferWord3);
    };
    auto fetch = [&](const char* base, int xw, bool ok, C (&dst)[S]) {
        const __amdgpu_buffer_rsrc_t rs = rsrc(base, xw, ok);
#pragma unroll
        for (int s = 0; s < S; ++s) dst[s] = load_c(rs, voff_ld[s], (C*)nullptr);
    };
    // x1 of sweep position p + k, |k| <= 3, from x1 of p (wrapped once on a
    // ring, whose N >= 3)
    const int Nwrap = periodic ? N : 0;
    auto shift = [&](int x, int k) {
        int y = x + k;
        y += y < 0 ? Nwrap : 0;
        y -= y >= N ? Nwrap : 0;
        return y;
    };
    int xc = periodic ? wrap3(it.x0, N) : it.x0;   // x1 of sweep position i (advanced per step)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        fetch(x_base, shift(xc, k), live(k), pre[k]);
        __builtin_amdgcn_sched_barrier(0);
    }

    const int total = nplanes + KT;
    const double wz = (zin && zout) ? 1.0 : 0.0;
    double nrm = 0.0;
    T tail = T(0);
    int buf = 0;

    for (int i0 = 0; i0 < total; i0 += 3) {
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int i = i0 + u;
            // ---- level 0: plane i enters; prefetch plane i + 3; bond above plane i
            {
                const int w = u;   // == i mod 3 (i0 is a multiple of 3)
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    yr[0][w][s] = FIRST ? pre[w][s].x * sc : pre[w][s].x;
                    yi[0][w][s] = FIRST ? pre[w][s].y * sc : pre[w][s].y;
                }
                fetch(x_base, shift(xc, 3), live(i + 3), pre[w]);
                // bond above plane i (0 at an open chain's first plane and past the sweep)
#pragma unroll
                for (int k = 0; k < KT; ++k) jq[k] = jq[k + 1];
                {
                    const bool has_up = live(i) && (periodic || xc > 0);
                    const T jup = Ju_t[has_up ? shift(xc, -1) : 0];   // index in range either way
                    jq[KT] = has_up ? jup : T(0);
                }
                // partial sum of plane i - 1, used when it completes (step i - 1 + KT)
                const int wb = m3(u - 1);
                if constexpr (FIRST || PROD) {
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        br[wb][s] = yr[0][wb][s];
                        bi[wb][s] = yi[0][wb][s];
                    }
                } else {
                    const __amdgpu_buffer_rsrc_t rs = rsrc(b_base, shift(xc, -1), live(i - 1));
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        const C v = load_c(rs, voff_ld[s], (C*)nullptr);
                        br[wb][s] = v.x;
                        bi[wb][s] = v.y;
                    }
                }
            }
            __syncthreads();   // edges published at the end of step i - 1
            const C* eb = &edge[buf][0][0][0][0];
            // ---- levels 1..KT: plane i - j
#pragma unroll
            for (int j = 1; j <= KT; ++j) {
                const int su = m3(u - j - 1), sm = m3(u - j), sd = m3(u - j + 1);
                const T Jup = jq[KT - j], Jdn = jq[KT - j + 1];
                const C up_e = eb[(((j - 1) * (W + 2) + wv) * 2 + 1) * 64 + lane];       // last row of wave w-1
                const C dn_e = eb[(((j - 1) * (W + 2) + wv + 2) * 2 + 0) * 64 + lane];   // first row of wave w+1
                const T cj = static_cast<T>(a.coef[j - 1]);
                const T cr = static_cast<T>(rot_re(j)) * cj, ci = static_cast<T>(rot_im(j)) * cj;
                const T pre_ = static_cast<T>(pp.cre[j - 1]), pim_ = static_cast<T>(pp.cim[j - 1]);
                const int p = i - j;
                const bool seed_ok = !LAST && j == KT && plane_out(p);
                __amdgpu_buffer_rsrc_t rs_seed;
                if constexpr (!LAST && !PROD)
                    if (j == KT) rs_seed = rsrc(q_base, shift(xc, -KT), seed_ok);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const T mr = yr[j - 1][sm][s], mi = yi[j - 1][sm][s];
                    const T ar = s > 0 ? yr[j - 1][sm][s > 0 ? s - 1 : 0] : up_e.x;
                    const T ai = s > 0 ? yi[j - 1][sm][s > 0 ? s - 1 : 0] : up_e.y;
                    const T br_ = s < S - 1 ? yr[j - 1][sm][s < S - 1 ? s + 1 : 0] : dn_e.x;
                    const T bi_ = s < S - 1 ? yi[j - 1][sm][s < S - 1 ? s + 1 : 0] : dn_e.y;
                    T hr, hi;
                    if constexpr (sizeof(T) == 4) {
                        stencil3_c64(hr, hi, dg[sm][s], mr, mi, yr[j - 1][su][s], yi[j - 1][su][s], yr[j - 1][sd][s],
                                     yi[j - 1][sd][s], ar, ai, br_, bi_, Jup, Jdn, jrow[s], jrow[s + 1], jl, jr);
                    } else {
                        hr = dg[sm][s] * mr;
                        hi = dg[sm][s] * mi;
                        hr = fma3(Jup, yr[j - 1][su][s], hr);
                        hi = fma3(Jup, yi[j - 1][su][s], hi);
                        hr = fma3(Jdn, yr[j - 1][sd][s], hr);
                        hi = fma3(Jdn, yi[j - 1][sd][s], hi);
                        hr = fma3(jrow[s], ar, hr);
                        hi = fma3(jrow[s], ai, hi);
                        hr = fma3(jrow[s + 1], br_, hr);
                        hi = fma3(jrow[s + 1], bi_, hi);
                        hr = fma3(jl, lane_from_left(mr), hr);
                        hi = fma3(jl, lane_from_left(mi), hi);
                        hr = fma3(jr, lane_from_right(mr), hr);
                        hi = fma3(jr, lane_from_right(mi), hi);
                    }
                    if (j < KT) {
                        yr[j][sm][s] = hr;
                        yi[j][sm][s] = hi;
                    }
                    // (-i)^j Y_j: odd j swaps the parts
                    const T xr = (j & 1) ? hi : hr, xi = (j & 1) ? hr : hi;
                    if constexpr (PROD) {
                        // c_j Y_j with complex c_j
                        if (j == 1) {
                            tr[sm][s] = fma3(pre_, hr, -(pim_ * hi));
                            ti[sm][s] = fma3(pre_, hi, pim_ * hr);
                        } else {
                            tr[sm][s] = fma3(pre_, hr, fma3(-pim_, hi, tr[sm][s]));
                            ti[sm][s] = fma3(pre_, hi, fma3(pim_, hr, ti[sm][s]));
                        }
                    } else if (j == 1) {
                        tr[sm][s] = cr * xr;
                        ti[sm][s] = ci * xi;
                    } else {
                        tr[sm][s] = fma3(cr, xr, tr[sm][s]);
                        ti[sm][s] = fma3(ci, xi, ti[sm][s]);
                    }
                    if constexpr (DO_TAIL) {
                        // |Y_K|^2 of this pass's last level (chained: the
                        // order's last term; product: the bound's base)
                        if (j == KT) {
                            const T m = (yout[s] && plane_out(p)) ? T(1) : T(0);
                            tail = fma3(m * hr, hr, fma3(m * hi, hi, tail));
                        }
                    }
                    if constexpr (!LAST && !PROD) {
                        if (j == KT) {
                            // Psi_{s+K} with its true phase, for the next pass
                            store_c(static_cast<T>(rot_re(KT)) * xr, static_cast<T>(rot_im(KT)) * xi, rs_seed,
                                    voff_st[s]);
                        }
                    }
                }
            }
            // ---- plane i - KT is complete
            {
                const int p = i - KT;
                const int w = m3(u - KT);
                const bool ok = plane_out(p);
                const __amdgpu_buffer_rsrc_t rs = rsrc(s_base, shift(xc, -KT), ok);
                double pn = 0.0;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const T orr = br[w][s] + tr[w][s];
                    const T oi = bi[w][s] + ti[w][s];
                    store_c(orr, oi, rs, voff_st[s]);
                    if constexpr (DO_NORM) {
                        const double dr = orr, di = oi;
                        pn = __builtin_fma(yout[s] ? dr : 0.0, dr, __builtin_fma(yout[s] ? di : 0.0, di, pn));
                    }
                }
                if constexpr (DO_NORM) {
                    if (ok) nrm += pn;
                }
            }
            // ---- diagonal of plane i (used from step i + 1 on; its slot held
            // plane i - 3, whose last use was level 3 of this step)
            {
                const int w = u;
                // (evaluated without branches: every index is in range either way)
                const bool xin = live(i);
                const int x1 = xin ? xc : 0;
                const T e1v = Eu_t[x1];
                const T e1 = xin ? e1v : T(0);
                const T u13 = (xin & ((x1 == zta) | (x1 == ztb))) ? Udt : T(0);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const T u12 = (xin & ((x1 == yta[s]) | (x1 == ytb[s]))) ? Udt : T(0);
                    dg[w][s] = drow[s] + (e1 + u12) + u13;
                }
            }
            // ---- publish the first and last rows of every level for step i + 1
            {
                buf ^= 1;
                C* ew = &edge[buf][0][0][0][0];
#pragma unroll
                for (int j = 0; j < KT; ++j) {
                    const int w = m3(u - j);   // level j holds plane i - j
                    C f, l;
                    f.x = yr[j][w][0];
                    f.y = yi[j][w][0];
                    l.x = yr[j][w][S - 1];
                    l.y = yi[j][w][S - 1];
                    ew[((j * (W + 2) + wv + 1) * 2 + 0) * 64 + lane] = f;
                    ew[((j * (W + 2) + wv + 1) * 2 + 1) * 64 + lane] = l;
                }
            }
            xc = shift(xc, 1);
        }
    }

    // ---- FP64 partials of the item: squared norm and last term
    if constexpr (DO_NORM || DO_TAIL) {
        __shared__ double red[2][W];
        const double n_w = wave_sum3(wz * nrm);
        const double t_w = wave_sum3(wz * (double)tail);
        if (lane == 0) {
            red[0][wv] = n_w;
            red[1][wv] = t_w;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double sn = 0.0, st = 0.0;
            for (int k = 0; k < W; ++k) {
                sn += red[0][k];
                st += red[1][k];
            }
            double f = a.tail_coef;
            if (PROD && !LAST) {
                // ||(dt H)^n psi|| <= x^(n - K) ||(dt H)^K psi||, x = dt G, from
                // the remainder factor r = (x / (n + 1)) / (1 - x / (n + 2))
                const int n = pp.order;
                const double r = rd.tail_factor_max;
                const double x = r / (1.0 / (n + 1) + r / (n + 2));
                double pw = 1.0;
                for (int k = pp.k_first; k < n; ++k) pw *= x;
                f = isfinite(r) ? f * pw : INFINITY;
            }
            if (DO_NORM) a.norm_part[home] = sn;
            if (DO_TAIL) a.tail_part[home] = st * f * f;
        }
    }
}

}  // namespace step3c_detail

namespace {
using Step3cFn = void (*)(Step3cArgs, Step3cProd);
// Compiled shapes: (dtype, terms per pass) -> kernel, rows per wave, waves.
struct Step3cShape {
    Step3cFn fn;
    int rows_per_wave;
    int waves;
};
Step3cShape select3c(int dtype, int K, bool first, bool last, bool prod) {
    using namespace step3c_detail;
#define CTQW_3C_P(T, KT, S, W, P)                                                                         \
    (first ? (last ? &step3c_kernel<T, KT, S, W, true, true, P> : &step3c_kernel<T, KT, S, W, true, false, P>) \
           : (last ? &step3c_kernel<T, KT, S, W, false, true, P> : &step3c_kernel<T, KT, S, W, false, false, P>))
#define CTQW_3C(T, KT, S, W) {prod ? CTQW_3C_P(T, KT, S, W, true) : CTQW_3C_P(T, KT, S, W, false), S, W}
    if (dtype == 1) {
        switch (K) {
            case 1: return CTQW_3C(double, 1, 4, 8);
            case 2: return CTQW_3C(double, 2, 3, 8);
            case 3: return CTQW_3C(double, 3, 2, 8);
            default: return {nullptr, 0, 0};
        }
    }
    switch (K) {
        case 1: return CTQW_3C(float, 1, 8, 8);
        case 2: return CTQW_3C(float, 2, 5, 8);
        case 3: return CTQW_3C(float, 3, 4, 8);
        default: return {nullptr, 0, 0};
    }
#undef CTQW_3C
#undef CTQW_3C_P
}
}  // namespace

int step3c_rows_per_block(int dtype, int K) {
    const Step3cShape sh = select3c(dtype, K, true, true, false);
    return sh.fn ? sh.rows_per_wave * sh.waves : 0;
}

namespace {
hipError_t launch3c(const Step3cArgs& a, const Step3cProd& pp, int dtype, int K, bool prod, hipStream_t stream) {
    const Step3cShape sh = select3c(dtype, K, a.first != 0, a.last != 0, prod);
    if (!sh.fn) return hipErrorInvalidValue;
    if (a.n_items <= 0) return hipSuccess;
    const int64_t per = ((int64_t)a.n_items + 7) / 8;
    const int64_t blocks = per * 8;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sh.fn, dim3((unsigned)blocks), dim3(64 * sh.waves), 0, stream, a, pp);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_step3c(const Step3cArgs& a, int dtype, int K, hipStream_t stream) {
    return launch3c(a, Step3cProd{}, dtype, K, false, stream);
}

hipError_t launch_step3c_prod(const Step3cArgs& a, const Step3cProd& pp, int dtype, int K, hipStream_t stream) {
    return launch3c(a, pp, dtype, K, true, stream);
}

}  // namespace ctqw
