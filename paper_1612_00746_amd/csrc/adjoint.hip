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
// One kernel does the work of a level: a row sweep (`sweep_kernel`) that
// computes y = cz z + s (-i) (dt H) (xs x) for every stored amplitude (s = +1
// for A, -1 for A^dagger) and, given v, accumulates Im <u| E |v> with
// u = xs x for every bond operator E (hopping across one bond, for every
// particle) and every site operator (the occupation of one node) into FP64
// sums.  A backward step is n - 1 such sweeps for v_1 .. v_{n-1} and n for
// the Horner chain, each contracting its input u_L with v_L while it forms
// u_{L-1} (lambda_k at L = 0); u_{n-1} = lambda / n! is the first sweep's
// scaled input, so no vector holds it.
//
// Work item: a band of 62 output columns of one realisation, held by one
// wave (one column per lane, one halo column on either side: the stencil and
// the bonds reach one column over), swept down the rows.  Rows q - 1, q,
// q + 1 of x and rows q, q + 1 of v are in registers; column neighbours come
// from the adjacent lanes.  Loads and stores run along rows, one amplitude
// per lane.
//
// Contractions.  Full grid (distinguishable particles; one particle is the
// one-row case): the column parts of bond c and site c are sums over the
// rows, kept per lane; the row parts of bond q and site q are sums over the
// columns, reduced across the wave at every row into one partial per band.
// Bosons are stored as the symmetric function phi(x1, x2) on x1 <= x2; the
// full-grid sums are then twice the column part, and the column part of
// bond b (pairs (q, b), (q, b + 1) over all q) splits into the stored pairs
// of row q <= b in columns b, b + 1 and, mirrored, the pairs of rows b,
// b + 1 in every column c >= b + 1: a horizontal part summed per lane and a
// vertical part summed per row, as for the full grid, with the vertical
// pairs and the row sites taken only where both entries are stored off the
// diagonal (site b: column b over rows q <= b, plus row b over columns
// c > b).  The stencil at a stored diagonal entry (q, q) reads its mirrored
// neighbours (q + 1, q) = (q, q + 1) and (q, q - 1) = (q - 1, q).
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

// Lane l receives lane l + 1's value (lane 63: 0) / lane l - 1's (lane 0: 0).
__device__ __forceinline__ float from_right(float x) { return __builtin_amdgcn_update_dpp(0.0f, x, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ double from_right(double x) { return __builtin_amdgcn_update_dpp(0.0, x, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ float from_left(float x) { return __builtin_amdgcn_update_dpp(0.0f, x, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ double from_left(double x) { return __builtin_amdgcn_update_dpp(0.0, x, 0x138, 0xF, 0xF, true); }

// Im(conj(u) v) in FP64.
template <typename T>
__device__ __forceinline__ double im_uv(T ur, T ui, T vr, T vi) {
    return (double)ur * (double)vi - (double)ui * (double)vr;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Im(conj(u) v) in the state's precision.
template <typename T>
__device__ __forceinline__ T im_t(T ur, T ui, T vr, T vi) {
    return fma(ur, vi, -(ui * vr));
}

// Eight values summed over the wave at once: each exchange step hands the
// partner the half of the values this lane does not keep (xor 32: four,
// xor 16: two, xor 8: one), then three steps sum the one value left.  Lane
// l ends with the total of value (l >> 3) (bits 5, 4, 3 of l pick it), in
// a fixed order of additions.  Ten shuffles instead of 48.
__device__ __forceinline__ double reduce8(const double (&v)[8], int lane) {
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0, b3 = (lane & 8) != 0;
    double w[4], x[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double send = b5 ? v[k] : v[k + 4];
        const double keep = b5 ? v[k + 4] : v[k];
        w[k] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double send = b4 ? w[k] : w[k + 2];
        const double keep = b4 ? w[k + 2] : w[k];
        x[k] = keep + __shfl_xor(send, 16, 64);
    }
    double y = (b3 ? x[1] : x[0]) + __shfl_xor(b3 ? x[0] : x[1], 8, 64);
    y += __shfl_xor(y, 4, 64);
    y += __shfl_xor(y, 2, 64);
    y += __shfl_xor(y, 1, 64);
    return y;
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRawBufferWord3 = 0x00020000;   // gfx9-family raw buffer, no format conversion
constexpr uint32_t kPastEnd = 0x80000000u;    // an offset past every row: loads read 0, stores drop

// One amplitude per lane through a buffer resource over a row.  Stores take
// a zero scalar offset (a 16-byte store reads its data registers after it
// issues; the compiler keeps the wait before the next write of them only
// when the scalar offset is not a register).
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
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, (int)off, 0, 0);
}
__device__ __forceinline__ void store_c(double re, double im, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    u32x4 v;
    v.x = (unsigned)__double2loint(re);
    v.y = (unsigned)__double2hiint(re);
    v.z = (unsigned)__double2loint(im);
    v.w = (unsigned)__double2hiint(im);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, 0);
}

// PER: ring; LAY: 0 one row (one particle), 1 full grid, 2 triangle (bosons).
template <typename T, bool CONTRACT, bool PER, int LAY>
__global__ void __launch_bounds__(64 * kSweepSegs) sweep_kernel(AdjSweepArgs a) {
    using C = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    const int r = blockIdx.y;
    const int w = blockIdx.x;
    const RealDev rd = a.reals[r];
    const int N = rd.N, rows = LAY == 0 ? 1 : rd.rows;
    // Bands are laid from the chain's end: band w of nbr outputs columns
    // [hi - 62, hi), hi = N - 62 (nbr - 1 - w), the first band the rest, so
    // that the narrow band sits where the triangle's columns are shortest.
    const int nbr = (N + kSweepOut - 1) / kSweepOut;
    if (w >= nbr) return;   // whole block, before the barrier
    const int hi_w = N - kSweepOut * (nbr - 1 - w);
    const int lo_w = max(0, hi_w - kSweepOut);
    const int lane = threadIdx.x & 63;
    const int seg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr bool periodic = PER;
    constexpr bool tri = LAY == 2;
    const T* Jc = reinterpret_cast<const T*>(a.Jt) + rd.param_off;
    const T* Ec = reinterpret_cast<const T*>(a.Et) + rd.param_off;
    const T* Jr = reinterpret_cast<const T*>(a.Jt) + rd.row_param_off;
    const T* Er = reinterpret_cast<const T*>(a.Et) + rd.row_param_off;
    const T Udt = static_cast<T>(rd.U * a.dt);
    const int want = (rd.flags & RF_NEAREST) ? 1 : 0;

    // this lane's column: window [lo_w - 1, lo_w + 63), output [lo_w, hi_w)
    const int c = lo_w - 1 + lane;
    const bool inb = periodic || (c >= 0 && c < N);
    const int cw = periodic ? wrapi(c, N) : (inb ? c : 0);
    const bool out = c >= lo_w && c < hi_w && lane > 0 && lane < 63;
    const T jl = (inb && (periodic || c > 0)) ? Jc[periodic ? wrapi(cw - 1, N) : cw - 1] : T(0);
    const T jr = (inb && (periodic || c < N - 1)) ? Jc[cw] : T(0);
    const T ec = inb ? Ec[cw] : T(0);
    const bool has_bond_c = periodic || c < N - 1;

    const C* X = reinterpret_cast<const C*>(a.x);
    const C* Z = reinterpret_cast<const C*>(a.z);
    const C* V = reinterpret_cast<const C*>(a.v);
    C* Y = reinterpret_cast<C*>(a.y);
    const T xs = static_cast<T>(a.xs), cz = static_cast<T>(a.cz), sg = static_cast<T>(a.sign);
    // lanes whose amplitude (q, c) is stored
    auto stored = [&](int q) { return inb && (!tri || cw >= q); };
    // Row q (wrapped on a ring) through a buffer resource over the row: its
    // first stored amplitude is (q, q) in the triangle, (q, 0) on the full
    // grid, and lane c reads column c; a lane without a stored amplitude,
    // or a row off the grid (resource length 0), reads 0.  No branches.
    const uint32_t row_bytes = (uint32_t)N * (uint32_t)sizeof(C);
    const uint32_t col_off = (uint32_t)cw * (uint32_t)sizeof(C);
    auto row_rsrc = [&](const C* base, int q, uint32_t& voff) {
        bool live = true;
        if (periodic) q = wrapi(q, rows);
        else {
            live = q >= 0 && q < rows;
            q = live ? q : 0;
        }
        // triangle row q holds columns q .. N - 1 from index q N - q (q + 1) / 2 + q
        const int64_t rb = tri ? (int64_t)q * N - ((int64_t)q * (q + 1)) / 2 : (int64_t)q * N;
        voff = stored(q) ? col_off : kPastEnd;
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<C*>(base) + rd.state_off + rb, 0,
                                                 live ? (int)row_bytes : 0, kRawBufferWord3);
    };
    auto ld = [&](const C* base, int q) -> C {
        if (!base) {
            C v;
            v.x = T(0);
            v.y = T(0);
            return v;
        }
        uint32_t voff;
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(base, q, voff);
        return load_c(rs, voff, (C*)nullptr);
    };
    // rows holding a stored amplitude of this window, split into one segment per wave
    const int q_end = tri ? min(rows, hi_w) : rows;
    const int q0 = (int)(((int64_t)q_end * seg) / kSweepSegs);
    const int q1 = (int)(((int64_t)q_end * (seg + 1)) / kSweepSegs);

    // Rows q - 1, q, q + 1 of x, q and q + 1 of v and q of z in registers; the
    // next kSweepAhead rows of each in a ring of loads in flight.
    C xm = ld(X, q0 - 1), x0 = ld(X, q0), xp = ld(X, q0 + 1);
    C v0 = CONTRACT ? ld(V, q0) : C{}, vp = CONTRACT ? ld(V, q0 + 1) : C{};
    C zq = ld(Z, q0);
    C xr[kSweepAhead], vr_[kSweepAhead], zr[kSweepAhead];
#pragma unroll
    for (int k = 0; k < kSweepAhead; ++k) {
        xr[k] = ld(X, q0 + 2 + k);
        vr_[k] = CONTRACT ? ld(V, q0 + 2 + k) : C{};
        zr[k] = ld(Z, q0 + 1 + k);
    }
    double bond_col = 0.0, site_col = 0.0;
    const double f = tri ? 2.0 : 1.0;
    double* gV = a.gV + ((int64_t)r * a.nb + w) * a.row_stride;
    double* gR = a.gR + ((int64_t)r * a.nb + w) * a.row_stride;
    for (int qb = q0; qb < q1; qb += kSweepAhead) {
        // row parts of the block's rows (bond q, site q per row), summed
        // over the lanes together after the block
        static_assert(2 * kSweepAhead == 8, "one reduce8 per block of rows");
        double rowpart[2 * kSweepAhead];
#pragma unroll
        for (int k = 0; k < kSweepAhead; ++k) {
            // rows past the segment run with every output off (no stores, no sums)
            const int q = qb + k;
            const bool live = q < q1;
            const T mr = xs * x0.x, mi = xs * x0.y;
            const T ur_ = xs * xm.x, ui_ = xs * xm.y;      // row q - 1
            const T dr_ = xs * xp.x, di_ = xs * xp.y;      // row q + 1
            const T rr = from_right(mr), ri = from_right(mi);
            const T lr = from_left(mr), li = from_left(mi);
            const bool diag = tri && cw == q;
            // neighbours below and to the left; mirrored on the stored diagonal
            const T br = diag ? rr : dr_, bi = diag ? ri : di_;
            const T ar = diag ? ur_ : lr, ai = diag ? ui_ : li;
            const int qr = periodic ? wrapi(q, rows) : min(q, rows - 1);   // in range either way
            const bool up = LAY != 0 && (periodic || q > 0);
            const bool dn = LAY != 0 && (periodic || q < rows - 1);
            const T Jup = up ? Jr[periodic ? wrapi(q - 1, rows) : min(max(q - 1, 0), rows - 1)] : T(0);
            const T Jdn = dn ? Jr[qr] : T(0);
            T d = Er[qr] + ec;
            if (LAY != 0) {
                int dd = q - cw;
                dd = dd < 0 ? -dd : dd;
                if (periodic && N - dd < dd) dd = N - dd;
                if (dd == want) d += Udt;
            }
            T hr = d * mr, hi = d * mi;
            hr = fma(Jup, ur_, hr);
            hi = fma(Jup, ui_, hi);
            hr = fma(Jdn, br, hr);
            hi = fma(Jdn, bi, hi);
            hr = fma(jl, ar, hr);
            hi = fma(jl, ai, hi);
            hr = fma(jr, rr, hr);
            hi = fma(jr, ri, hi);
            const bool st = live && out && stored(q);
            {
                // s (-i)(hr + i hi) = s (hi - i hr); lanes without an output drop the store
                uint32_t voff;
                const __amdgpu_buffer_rsrc_t rs = row_rsrc(Y, q, voff);
                store_c(fma(cz, zq.x, sg * hi), fma(cz, zq.y, -sg * hr), rs, st ? voff : kPastEnd);
            }
            if constexpr (CONTRACT) {
                // Im conj(u) v in the state's precision per pair, summed in FP64;
                // every lane computes, lanes without an output add zeros
                const T vr = from_right(v0.x), vi = from_right(v0.y);
                const T s0 = im_t(mr, mi, v0.x, v0.y);
                const T hb = im_t(mr, mi, vr, vi) + im_t(rr, ri, v0.x, v0.y);
                site_col += st ? (double)s0 : 0.0;
                bond_col += (st && has_bond_c) ? (double)hb : 0.0;
                const T vb = im_t(mr, mi, vp.x, vp.y) + im_t(dr_, di_, v0.x, v0.y);
                rowpart[2 * k] = (st && dn && (!tri || cw >= q + 1)) ? (double)vb : 0.0;
                rowpart[2 * k + 1] = (st && !diag) ? (double)s0 : 0.0;
                v0 = vp;
                vp = vr_[k];
                vr_[k] = ld(V, q + 2 + kSweepAhead);
            }
            xm = x0;
            x0 = xp;
            xp = xr[k];
            xr[k] = ld(X, q + 2 + kSweepAhead);
            zq = zr[k];
            zr[k] = ld(Z, q + 1 + kSweepAhead);
        }
        if constexpr (CONTRACT) {
            if (LAY != 0) {
                // lane 8 j ends with the wave's sum of rowpart[j]
                const double t = reduce8(rowpart, lane);
                const int j = lane >> 3;
                const int q = qb + (j >> 1);
                if ((lane & 7) == 0 && q < q1) {
                    if (j & 1) gR[q] += f * t;
                    else gV[q] += f * t;
                }
            }
        }
    }
    if constexpr (CONTRACT) {
        // column parts of the segments, summed in segment order
        __shared__ double part[2][kSweepSegs][64];
        part[0][seg][lane] = bond_col;
        part[1][seg][lane] = site_col;
        __syncthreads();
        if (seg == 0 && out) {
            double sb = 0.0, ss = 0.0;
#pragma unroll
            for (int k = 0; k < kSweepSegs; ++k) {
                sb += part[0][k][lane];
                ss += part[1][k][lane];
            }
            const int64_t o = a.site_off[r] + cw;
            a.gJ[o] += f * sb;
            a.gE[o] += f * ss;
        }
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

hipError_t launch_adj_sweep(const AdjSweepArgs& a, hipStream_t s) {
    if (a.R > 65535 || a.nb < 1 || a.nb > 65535) return hipErrorInvalidValue;
    const dim3 g((unsigned)a.nb, (unsigned)a.R);
    const bool con = a.v != nullptr;
    if (a.layout < 0 || a.layout > 2) return hipErrorInvalidValue;
    using Fn = void (*)(AdjSweepArgs);
#define CTQW_SWEEP(T, C, PER)                                                                     \
    (a.layout == 0 ? (Fn)&sweep_kernel<T, C, PER, 0>                                              \
                   : (a.layout == 1 ? (Fn)&sweep_kernel<T, C, PER, 1> : (Fn)&sweep_kernel<T, C, PER, 2>))
    Fn fn;
    if (a.dtype == 1) {
        fn = con ? (a.periodic ? CTQW_SWEEP(double, true, true) : CTQW_SWEEP(double, true, false))
                 : (a.periodic ? CTQW_SWEEP(double, false, true) : CTQW_SWEEP(double, false, false));
    } else {
        fn = con ? (a.periodic ? CTQW_SWEEP(float, true, true) : CTQW_SWEEP(float, true, false))
                 : (a.periodic ? CTQW_SWEEP(float, false, true) : CTQW_SWEEP(float, false, false));
    }
#undef CTQW_SWEEP
    hipLaunchKernelGGL(fn, g, dim3(64 * kSweepSegs), 0, s, a);
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
    hipLaunchKernelGGL(adj_reduce_kernel, dim3((unsigned)a.N + 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ctqw
