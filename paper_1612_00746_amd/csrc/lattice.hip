// One particle on a two-dimensional lattice (q = 2: Sec. 2, a node couples to
// its four lattice neighbours; the capacity example of Sec. 3), R statically
// noisy realisations, each with its own coupling on every bond and its own
// on-site energy on every node (Eq. 1 with the noise drawn per bond and per
// node), advanced by the truncated Taylor series of exp(-i H dt) (Eqs. 5-7,
// Alg. 3) with all n terms of a step in one pass over the state.
//
// The state of realisation r is psi[r][y][x] (x fastest).  A work item is a
// band of 64 columns (one per lane) of one realisation, swept over the rows
// y with an n-level register pipeline, as for two walkers on a chain: at
// sweep step i row i enters level 0, level j forms Y_j = (dt H) Y_(j-1) on
// row i - j from level j - 1's rows i - j - 1, i - j, i - j + 1, and row
// i - n is complete.  Unlike the chain, the couplings vary along both axes,
// so every row brings its own per-lane tables -- the bond to the right, the
// bond below and the on-site energy, dt-scaled -- which ride with the row
// through the pipeline in a ring of registers (the bond to the left of a
// column is the right bond of the lane before, taken once per row).
//   (dt H y)(x, y) = e(x, y) m + jd(x, y - 1) u + jd(x, y) d + jr(x - 1, y) l + jr(x, y) r
// (m: this amplitude; u, d: the rows above and below; l, r: the adjacent
// lanes).  The terms (-i)^j Y_j / j! are summed apart from psi and added to
// it once, when the row completes; the squared FP64 norm of the new state
// is reduced per item.  Bands overlap by n columns (the halo); a ring in y
// is swept n rows early and late.
//
// HBM bytes per node and step: read psi and the three tables, write psi
// (complex64: 8 + 12 + 8 = 28 B), times the band overlap on the reads.
#include "../../include/ctqw.h"
#include "ctqw_internal.hpp"

#include <algorithm>
#include <vector>

namespace ctqw {
namespace lattice_detail {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kWord3 = 0x00020000;            // gfx9-family raw buffer, no format conversion
constexpr uint32_t kPastEnd = 0x80000000u;    // an offset past every row: loads read 0, stores drop

__device__ __forceinline__ float lane_left(float x) { return __builtin_amdgcn_update_dpp(0.0f, x, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ double lane_left(double x) { return __builtin_amdgcn_update_dpp(0.0, x, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ float lane_right(float x) { return __builtin_amdgcn_update_dpp(0.0f, x, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ double lane_right(double x) { return __builtin_amdgcn_update_dpp(0.0, x, 0x130, 0xF, 0xF, true); }

__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float2 load_c(__amdgpu_buffer_rsrc_t rs, uint32_t off, float2*) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}
__device__ __forceinline__ double2 load_c(__amdgpu_buffer_rsrc_t rs, uint32_t off, double2*) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    return make_double2(__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z));
}
__device__ __forceinline__ float load_r(__amdgpu_buffer_rsrc_t rs, uint32_t off, float*) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
}
__device__ __forceinline__ double load_r(__amdgpu_buffer_rsrc_t rs, uint32_t off, double*) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
    return __hiloint2double((int)v.y, (int)v.x);
}
// Stores take a zero scalar offset (a 16-byte store reads its data registers
// after it issues; the compiler keeps the wait before the next write of
// them only when the scalar offset is not a register).
__device__ __forceinline__ void store_c(float re, float im, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x2 v;
    v.x = __float_as_uint(re);
    v.y = __float_as_uint(im);
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, (int)off, 0, 2);
}
__device__ __forceinline__ void store_c(double re, double im, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x4 v;
    v.x = (unsigned)__double2loint(re);
    v.y = (unsigned)__double2hiint(re);
    v.z = (unsigned)__double2loint(im);
    v.w = (unsigned)__double2hiint(im);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, 2);
}

// rows in flight: n levels, the row above the deepest one and the row entering
__host__ __device__ constexpr int ring_rows(int nt) { return ((nt + 4) / 3) * 3; }   // >= nt + 2, a multiple of 3
__host__ __device__ constexpr int mpos(int x, int w) { return ((x % w) + w) % w; }
__host__ __device__ constexpr double inv_fact(int j) {
    double f = 1.0;
    for (int k = 2; k <= j; ++k) f *= k;
    return 1.0 / f;
}
// (-i)^j = (sr, si) applied after the swap of roles: for odd j the real part
// of (-i)^j y is si_j Im y, the imaginary part sr_j Re y.
__host__ __device__ constexpr double rot_re(int j) { return (j % 4 == 0 || j % 4 == 1) ? 1.0 : -1.0; }
__host__ __device__ constexpr double rot_im(int j) { return (j % 4 == 0 || j % 4 == 3) ? 1.0 : -1.0; }

// Band b of 64 columns with a halo of h: window start w0, output [lo, hi).
// Open chain: the first window starts at column 0 and every later one h
// columns before its output; a window that reaches the end outputs up to
// it.  Ring: every window starts h columns before its output.
__host__ __device__ inline void band_geom(int b, int Lx, int h, bool periodic, int* w0, int* lo, int* hi) {
    const int step = 64 - 2 * h;
    if (periodic) {
        *lo = b * step;
        *w0 = *lo - h;
        *hi = (*lo + step < Lx) ? *lo + step : Lx;
    } else {
        *lo = b == 0 ? 0 : 64 - h + (b - 1) * step;
        *w0 = b == 0 ? 0 : *lo - h;
        *hi = (*w0 + 64 >= Lx) ? Lx : *w0 + 64 - h;
    }
}
// Bands up to the one whose output reaches the end of the chain.
__host__ inline int band_count(int Lx, int h, bool periodic) {
    if (64 - 2 * h <= 0) return 0;
    for (int b = 0;; ++b) {
        int w0, lo, hi;
        band_geom(b, Lx, h, periodic, &w0, &lo, &hi);
        if (hi >= Lx) return b + 1;
    }
}

__device__ __forceinline__ int wrapi(int x, int n) { int r = x % n; return r < 0 ? r + n : r; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// dt-scaled tables with the open boundaries' missing bonds set to zero.
template <typename T>
__global__ void __launch_bounds__(256) scale_tables_kernel(LatticeArgs a) {
    const int64_t n = (int64_t)a.Lx * a.Ly;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n * a.R) return;
    const int x = (int)((k % n) % a.Lx), y = (int)((k % n) / a.Lx);
    const T* jx = static_cast<const T*>(a.Jx);
    const T* jy = static_cast<const T*>(a.Jy);
    const T* e = static_cast<const T*>(a.eps);
    T* jr = static_cast<T*>(a.tab);
    T* jd = jr + n * a.R;
    T* es = jd + n * a.R;
    const T dt = static_cast<T>(a.dt);
    jr[k] = (a.px || x < a.Lx - 1) ? dt * jx[k] : T(0);
    jd[k] = (a.py || y < a.Ly - 1) ? dt * jy[k] : T(0);
    es[k] = dt * e[k];
}

template <typename T, int NT>
__global__ void __launch_bounds__(256) lattice_kernel(LatticeArgs a) {
    using C = typename Cplx<T>::type;
    constexpr int WA = ring_rows(NT);
    constexpr int PF = 3;   // rows fetched ahead
    static_assert(WA % PF == 0, "the prefetch ring must tile the unrolled block");
    const int lane = threadIdx.x & 63;
    const int item = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (item >= a.n_items) return;   // whole wave; the kernel has no barrier
    const int r = __builtin_amdgcn_readfirstlane(item / a.nb);
    const int b = __builtin_amdgcn_readfirstlane(item % a.nb);
    const int Lx = a.Lx, Ly = a.Ly;
    const bool px = a.px != 0, py = a.py != 0;
    int w0, lo, hi;
    band_geom(b, Lx, NT, px, &w0, &lo, &hi);
    const int64_t nodes = (int64_t)Lx * Ly;

    // this lane's column
    const int c = w0 + lane;
    const bool inb = px || (c >= 0 && c < Lx);
    const int cw = px ? wrapi(c, Lx) : (inb ? c : 0);
    const bool outv = inb && c >= lo && c < hi;
    const uint32_t off_c = inb ? (uint32_t)cw * (uint32_t)sizeof(C) : kPastEnd;
    const uint32_t off_t = inb ? (uint32_t)cw * (uint32_t)sizeof(T) : kPastEnd;
    const uint32_t off_o = outv ? (uint32_t)cw * (uint32_t)sizeof(C) : kPastEnd;

    const C* in = static_cast<const C*>(a.psi_in) + r * nodes;
    C* out = static_cast<C*>(a.psi_out) + r * nodes;
    const T* jr_t = static_cast<const T*>(a.tab) + r * nodes;
    const T* jd_t = jr_t + nodes * a.R;
    const T* e_t = jd_t + nodes * a.R;
    const int row0 = py ? -NT : 0;
    const int nrows = py ? Ly + 2 * NT : Ly;
    const uint32_t row_c = (uint32_t)Lx * (uint32_t)sizeof(C);
    const uint32_t row_t = (uint32_t)Lx * (uint32_t)sizeof(T);

    // Row i of the sweep through buffer resources (length 0 past the sweep)
    C pre[PF];
    T pre_jr[PF], pre_jd[PF], pre_e[PF];
    auto fetch = [&](int i, int slot) {
        const bool live = i < nrows;
        const int qa = row0 + i;
        const int qw = py ? wrapi(qa, Ly) : (live ? qa : 0);
        const int64_t base = (int64_t)qw * Lx;
        const __amdgpu_buffer_rsrc_t rc =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<C*>(in + base), 0, live ? (int)row_c : 0, kWord3);
        const __amdgpu_buffer_rsrc_t r1 =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(jr_t + base), 0, live ? (int)row_t : 0, kWord3);
        const __amdgpu_buffer_rsrc_t r2 =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(jd_t + base), 0, live ? (int)row_t : 0, kWord3);
        const __amdgpu_buffer_rsrc_t r3 =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(e_t + base), 0, live ? (int)row_t : 0, kWord3);
        pre[slot] = load_c(rc, off_c, (C*)nullptr);
        pre_jr[slot] = load_r(r1, off_t, (T*)nullptr);
        pre_jd[slot] = load_r(r2, off_t, (T*)nullptr);
        pre_e[slot] = load_r(r3, off_t, (T*)nullptr);
    };

    T yr[NT][3], yi[NT][3];             // Y_j rows, j < NT (planes modulo 3)
    T pr[WA], pi[WA];                   // psi of the rows in flight
    T tr[WA], ti[WA];                   // their summed terms
    T er[WA], jrr[WA], jlr[WA], jdr[WA];   // their tables
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int s = 0; s < 3; ++s) yr[j][s] = yi[j][s] = T(0);
#pragma unroll
    for (int w = 0; w < WA; ++w) pr[w] = pi[w] = tr[w] = ti[w] = er[w] = jrr[w] = jlr[w] = jdr[w] = T(0);
#pragma unroll
    for (int s = 0; s < PF; ++s) {
        fetch(s, s);
        __builtin_amdgcn_sched_barrier(0);
    }

    double nrm = 0.0;
    const int total = nrows + NT;
    for (int i0 = 0; i0 < total; i0 += WA) {
#pragma unroll
        for (int u = 0; u < WA; ++u) {
            const int i = i0 + u;
            // ---- level 0: row i enters (zero past the sweep)
            {
                const int s = u % 3, sp = u % PF, w = u;
                yr[0][s] = pre[sp].x;
                yi[0][s] = pre[sp].y;
                pr[w] = pre[sp].x;
                pi[w] = pre[sp].y;
                tr[w] = ti[w] = T(0);
                er[w] = pre_e[sp];
                jrr[w] = pre_jr[sp];
                jlr[w] = lane_left(pre_jr[sp]);
                jdr[w] = pre_jd[sp];
                fetch(i + PF, sp);
            }
            // ---- levels 1..NT: row i - j
#pragma unroll
            for (int j = 1; j <= NT; ++j) {
                const int su = mpos(u - j - 1, 3), sm = mpos(u - j, 3), sd = mpos(u - j + 1, 3);
                const int w = mpos(u - j, WA), wu = mpos(u - j - 1, WA);
                const T mr = yr[j - 1][sm], mi = yi[j - 1][sm];
                T hr = er[w] * mr, hi = er[w] * mi;
                hr = fmat(jdr[wu], yr[j - 1][su], hr);
                hi = fmat(jdr[wu], yi[j - 1][su], hi);
                hr = fmat(jdr[w], yr[j - 1][sd], hr);
                hi = fmat(jdr[w], yi[j - 1][sd], hi);
                hr = fmat(jlr[w], lane_left(mr), hr);
                hi = fmat(jlr[w], lane_left(mi), hi);
                hr = fmat(jrr[w], lane_right(mr), hr);
                hi = fmat(jrr[w], lane_right(mi), hi);
                if (j < NT) {
                    yr[j][sm] = hr;
                    yi[j][sm] = hi;
                }
                // (-i)^j Y_j / j!: odd j swaps the parts
                const T cr = static_cast<T>(rot_re(j) * inv_fact(j)), ci = static_cast<T>(rot_im(j) * inv_fact(j));
                tr[w] = fmat(cr, (j & 1) ? hi : hr, tr[w]);
                ti[w] = fmat(ci, (j & 1) ? hr : hi, ti[w]);
            }
            // ---- row i - NT is complete
            {
                const int q = i - NT;
                const int w = mpos(u - NT, WA);
                const int qa = row0 + q;
                const bool ok = q >= 0 && qa >= 0 && qa < Ly;
                const T orr = pr[w] + tr[w], oi = pi[w] + ti[w];
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    out + (int64_t)(ok ? qa : 0) * Lx, 0, ok ? (int)row_c : 0, kWord3);
                store_c(orr, oi, rs, off_o);
                const double dr = orr, di = oi;
                const double wgt = (ok && outv) ? 1.0 : 0.0;
                nrm = __builtin_fma(wgt * dr, dr, __builtin_fma(wgt * di, di, nrm));
            }
        }
    }
    nrm = wave_sum(nrm);
    if (lane == 0) a.norm_part[item] = nrm;
}

// out[r] = sum over the bands of realisation r of their partials, in band order.
__global__ void lattice_norm_kernel(const double* part, int32_t nb, int32_t R, double* out) {
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= R) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)r * nb + b];
    out[r] = s;
}

using KernelFn = void (*)(LatticeArgs);
template <typename T, int... Ns>
KernelFn pick(int order, std::integer_sequence<int, Ns...>) {
    KernelFn fn = nullptr;
    ((fn = (order == Ns + 1) ? &lattice_kernel<T, Ns + 1> : fn), ...);
    return fn;
}

}  // namespace lattice_detail

int lattice_max_order(int dtype) { return dtype == 1 ? kLatticeMaxOrderC128 : kLatticeMaxOrderC64; }

hipError_t launch_lattice_scale(const LatticeArgs& a, int dtype, hipStream_t s) {
    using namespace lattice_detail;
    const int64_t n = (int64_t)a.Lx * a.Ly * a.R;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (dtype == 1) hipLaunchKernelGGL(scale_tables_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(scale_tables_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lattice_step(const LatticeArgs& a, int dtype, int order, hipStream_t s) {
    using namespace lattice_detail;
    KernelFn fn = dtype == 1 ? pick<double>(order, std::make_integer_sequence<int, kLatticeMaxOrderC128>{})
                             : pick<float>(order, std::make_integer_sequence<int, kLatticeMaxOrderC64>{});
    if (!fn) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((a.n_items + 3) / 4);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_lattice_norms(const double* part, int32_t nb, int32_t R, double* out, hipStream_t s) {
    hipLaunchKernelGGL(lattice_detail::lattice_norm_kernel, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s,
                       part, nb, R, out);
    return hipGetLastError();
}

}  // namespace ctqw

// ------------------------------------------------------------------ C ABI

namespace {

using namespace ctqw;

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct LatticeLayout {
    int64_t state = 0, tab = 0, part = 0, total = 0;
};

ctqw_status lat_fail(ctqw_status st, const char* msg) { return (ctqw_status)report_error(st, msg); }

ctqw_status lattice_layout(int32_t Lx, int32_t Ly, int32_t R, int32_t dtype, int32_t order, int32_t periodic_x,
                           LatticeLayout* lay, int32_t* n_bands) {
    if (Lx < 1 || Ly < 1 || R < 1) return lat_fail(CTQW_ERR_INVALID_ARG, "need Lx, Ly, R >= 1");
    if (periodic_x && Lx < 3) return lat_fail(CTQW_ERR_INVALID_ARG, "a ring needs at least 3 nodes");
    if (dtype != CTQW_C64 && dtype != CTQW_C128) return lat_fail(CTQW_ERR_INVALID_ARG, "unknown dtype");
    const int maxo = lattice_max_order(dtype == CTQW_C128 ? 1 : 0);
    if (order < 1 || order > maxo) {
        char m[128];
        snprintf(m, sizeof m, "order must be in 1..%d for this dtype (got %d)", maxo, order);
        return lat_fail(order < 1 ? CTQW_ERR_INVALID_ARG : CTQW_ERR_UNSUPPORTED, m);
    }
    if ((int64_t)Lx * Ly * R > ((int64_t)1 << 31) / 3)
        return lat_fail(CTQW_ERR_UNSUPPORTED, "lattice tables beyond 2^31 entries");
    if ((int64_t)Lx * (dtype == CTQW_C128 ? 16 : 8) > ((int64_t)1 << 30))
        return lat_fail(CTQW_ERR_UNSUPPORTED, "rows beyond 2^30 bytes");
    const int nb = lattice_detail::band_count(Lx, order, periodic_x != 0);
    if (nb <= 0) return lat_fail(CTQW_ERR_UNSUPPORTED, "order too deep for the band width");
    if ((int64_t)nb * R > INT32_MAX / 2) return lat_fail(CTQW_ERR_UNSUPPORTED, "too many work items");
    const int64_t n = (int64_t)Lx * Ly * R;
    const int64_t csz = dtype == CTQW_C128 ? 16 : 8, rsz = csz / 2;
    LatticeLayout l;
    l.state = 0;
    l.tab = align256(l.state + n * csz);
    l.part = align256(l.tab + 3 * n * rsz);
    l.total = align256(l.part + (int64_t)nb * R * 8);
    *lay = l;
    if (n_bands) *n_bands = nb;
    return CTQW_OK;
}

}  // namespace

extern "C" ctqw_status ctqw_lattice_workspace(int32_t Lx, int32_t Ly, int32_t R, int32_t dtype, int32_t order,
                                              int32_t periodic_x, int64_t* bytes) {
    if (!bytes) return lat_fail(CTQW_ERR_INVALID_ARG, "NULL argument");
    LatticeLayout l;
    const ctqw_status st = lattice_layout(Lx, Ly, R, dtype, order, periodic_x, &l, nullptr);
    if (st != CTQW_OK) return st;
    *bytes = l.total;
    return CTQW_OK;
}

extern "C" ctqw_status ctqw_lattice_evolve(int32_t Lx, int32_t Ly, int32_t periodic_x, int32_t periodic_y, int32_t R,
                                           const void* Jx, const void* Jy, const void* eps, int32_t dtype, double dt,
                                           int32_t order, int64_t n_steps, void* psi, void* workspace,
                                           int64_t workspace_bytes, double* norms, void* hip_stream) {
    LatticeLayout l;
    int32_t nb = 0;
    ctqw_status st = lattice_layout(Lx, Ly, R, dtype, order, periodic_x, &l, &nb);
    if (st != CTQW_OK) return st;
    if (!Jx || !Jy || !eps || !psi || !workspace) return lat_fail(CTQW_ERR_INVALID_ARG, "NULL argument");
    if (periodic_y && Ly < 3) return lat_fail(CTQW_ERR_INVALID_ARG, "a ring needs at least 3 nodes");
    if (!std::isfinite(dt)) return lat_fail(CTQW_ERR_INVALID_ARG, "dt must be finite");
    if (n_steps < 0) return lat_fail(CTQW_ERR_INVALID_ARG, "n_steps must be >= 0");
    if (workspace_bytes < l.total) return lat_fail(CTQW_ERR_INVALID_ARG, "workspace too small");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return lat_fail(CTQW_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int d = dtype == CTQW_C128 ? 1 : 0;
    char* ws = static_cast<char*>(workspace);
    auto hip_fail = [](hipError_t e) { return lat_fail(CTQW_ERR_DEVICE, hipGetErrorString(e)); };
    hipError_t e;
    LatticeArgs a{};
    a.Jx = Jx;
    a.Jy = Jy;
    a.eps = eps;
    a.tab = ws + l.tab;
    a.norm_part = reinterpret_cast<double*>(ws + l.part);
    a.Lx = Lx;
    a.Ly = Ly;
    a.R = R;
    a.px = periodic_x != 0;
    a.py = periodic_y != 0;
    a.nb = nb;
    a.n_items = nb * R;
    a.dt = dt;
    if ((e = launch_lattice_scale(a, d, s)) != hipSuccess) return hip_fail(e);
    const int64_t bytes = (int64_t)Lx * Ly * R * (d ? 16 : 8);
    void* buf[2] = {psi, ws + l.state};
    for (int64_t k = 0; k < n_steps; ++k) {
        a.psi_in = buf[k & 1];
        a.psi_out = buf[(k + 1) & 1];
        if ((e = launch_lattice_step(a, d, order, s)) != hipSuccess) return hip_fail(e);
        if (norms && (e = launch_lattice_norms(a.norm_part, nb, R, norms + k * (int64_t)R, s)) != hipSuccess)
            return hip_fail(e);
    }
    if (n_steps & 1) {
        if ((e = hipMemcpyAsync(psi, ws + l.state, bytes, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(e);
    }
    return CTQW_OK;
}
