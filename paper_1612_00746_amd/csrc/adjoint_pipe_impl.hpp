// The K-level adjoint pass (see adjoint_pipe.hpp for what it computes).
//
// Per wave: one band of columns (one per lane, K halo lanes on either side)
// and one row segment, swept from K rows before the segment to K rows after
// it.  At sweep step i:
//   * level 0: row i of X (or of Z when the pass starts from Z itself)
//     enters, scaled by xs; rows past the sweep enter as zero;
//   * level l = 1 .. K: row i - l of Y_l from level l - 1's rows
//     i - l - 1, i - l, i - l + 1 (a 3-row register window per level), plus
//     cz_l times row i - l of Z; lanes without a stored amplitude (off the
//     chain, the triangle's lower part) are held at zero; stored if
//     y[l - 1] is set; and, for the Horner passes, level l's input row
//     contracted with rows i - l, i - l + 1 of v[l - 1];
//   * the row parts of row i - K (its last contribution came from level K)
//     join a batch of three rows, which is summed over the wave at once.
// Everything that follows a row down the levels -- its Z row, the partner
// rows of v (fetched three steps ahead), its row parts -- rides in a shift
// register with one stage per level, so the sweep needs no unrolling beyond
// the three steps of the row windows (a longer unroll let the compiler keep
// every step's row addresses in scalar registers at once, which spilled).
// Contractions.  Full grid (distinguishable particles; one particle is the
// one-row case): the column parts of bond c and site c are sums over the
// rows, kept per lane; the row parts of bond q and site q are sums over the
// columns, reduced across the wave for three rows at a time into one
// partial per band.
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
#pragma once

#include "adjoint_common.hpp"
#include "adjoint_pipe.hpp"

#include <type_traits>

namespace ctqw {
namespace adj_pipe {

using namespace adj;

__host__ __device__ constexpr int mpos(int x, int w) { return ((x % w) + w) % w; }

template <typename T, int K, int LAY, bool PER, bool CON>
__global__ void __launch_bounds__(64 * kSweepSegs, 2) pipe_kernel(AdjPipeArgs a) {
    using C = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    constexpr int W = 64 - 2 * K;          // output columns per band
    static_assert(K >= 1 && K <= kPipeMaxLevels, "levels per pass");
    static_assert(!(PER && LAY == 2), "no triangle on a ring");
    constexpr bool periodic = PER;          // columns on a ring
    constexpr bool rper = PER && LAY != 0;  // rows on a ring (one particle: a single row)
    constexpr bool tri = LAY == 2;

    const int r = blockIdx.y;
    const int w = blockIdx.x;
    const RealDev rd = a.reals[r];
    const int N = rd.N, rows = LAY == 0 ? 1 : rd.rows;
    // Bands are laid from the chain's end: band w outputs [hi - W, hi),
    // hi = N - W (nbr - 1 - w), the first band the rest.
    const int nbr = (N + W - 1) / W;
    if (w >= nbr) return;   // whole block, before the barrier
    const int hi_w = N - W * (nbr - 1 - w);
    const int lo_w = max(0, hi_w - W);
    const int lane = threadIdx.x & 63;
    const int seg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const T* Jc = reinterpret_cast<const T*>(a.Jt) + rd.param_off;
    const T* Ec = reinterpret_cast<const T*>(a.Et) + rd.param_off;
    const T* Jr = reinterpret_cast<const T*>(a.Jt) + rd.row_param_off;
    const T* Er = reinterpret_cast<const T*>(a.Et) + rd.row_param_off;
    const T Udt = static_cast<T>(rd.U * a.dt);
    const int want = (rd.flags & RF_NEAREST) ? 1 : 0;
    const T sg = static_cast<T>(a.sign);
    const T xs = static_cast<T>(a.xs);

    // this lane's column: window [lo_w - K, lo_w - K + 64), output [lo_w, hi_w)
    const int c = lo_w - K + lane;
    const bool inb = periodic || (c >= 0 && c < N);
    const int cw = periodic ? wrapi(c, N) : (inb ? c : 0);
    const bool out = c >= lo_w && c < hi_w;
    const T jl = (inb && (periodic || c > 0)) ? Jc[periodic ? wrapi(cw - 1, N) : cw - 1] : T(0);
    const T jr = (inb && (periodic || c < N - 1)) ? Jc[cw] : T(0);
    const T ec = inb ? Ec[cw] : T(0);
    const bool has_bond_c = periodic || c < N - 1;
    auto stored = [&](int q) { return inb && (!tri || cw >= q); };

    // rows holding a stored amplitude of this window, split into one segment
    // per wave; the sweep runs K rows beyond the segment on either side
    const int q_end = tri ? min(rows, hi_w) : rows;
    const int q0 = (int)(((int64_t)q_end * seg) / kSweepSegs);
    const int q1 = (int)(((int64_t)q_end * (seg + 1)) / kSweepSegs);
    const int s_lo = rper ? q0 - K : max(0, q0 - K);
    const int s_hi = rper ? q1 + K : min(rows, q1 + K);
    const int nsweep = q1 > q0 ? s_hi - s_lo : 0;
    const int o_lo = q0 - s_lo, o_hi = q1 - s_lo;   // output rows, as sweep steps

    const uint32_t col_off = (uint32_t)cw * (uint32_t)sizeof(C);
    // grid row of sweep step s (wrapped on a ring)
    auto grid_row = [&](int s) { return rper ? wrapi(s_lo + s, rows) : s_lo + s; };
    // One buffer resource per array over this realisation's amplitudes (the
    // launcher keeps them under 2^31 bytes), the row in the per-lane offset:
    // a 32-bit offset per access instead of a resource per row.  Lanes
    // without a stored amplitude, and rows outside the sweep, take an offset
    // past the end: loads read 0 and stores are dropped.
    const uint32_t real_bytes =
        (uint32_t)(tri ? N * (N + 1) / 2 : rows * N) * (uint32_t)sizeof(C);
    auto arr_rsrc = [&](const void* base) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<C*>(reinterpret_cast<const C*>(base)) + rd.state_off, 0,
                                                 base ? (int)real_bytes : 0, kRawBufferWord3);
    };
    auto lane_off = [&](int s) -> uint32_t {
        int q = s_lo + s;
        const bool live = s >= 0 && s < nsweep;
        if (rper) q = wrapi(q, rows);
        q = live ? q : 0;
        const uint32_t rowb = (uint32_t)(tri ? q * N - (q * (q + 1)) / 2 : q * N) * (uint32_t)sizeof(C);
        return (live && stored(q)) ? rowb + col_off : kPastEnd;
    };
    auto ldrow = [&](const __amdgpu_buffer_rsrc_t rs, int s) -> C { return load_c(rs, lane_off(s), (C*)nullptr); };

    // The Horner passes (CON) add Z to every level; the forward passes have none.
    const bool x_is_z = CON && a.x == a.z;
    const __amdgpu_buffer_rsrc_t X = arr_rsrc(x_is_z ? nullptr : a.x);
    const __amdgpu_buffer_rsrc_t Z = arr_rsrc(CON ? a.z : nullptr);
    // stored levels: every level of a forward pass, the last of a Horner pass
    __amdgpu_buffer_rsrc_t Y[K], V[CON ? K : 1];
#pragma unroll
    for (int l = 0; l < K; ++l) Y[l] = arr_rsrc((!CON || l == K - 1) ? a.y[l] : nullptr);
    if constexpr (CON) {
#pragma unroll
        for (int l = 0; l < K; ++l) V[l] = arr_rsrc(a.v[l]);
    }

    T yr[K][3], yi[K][3];          // levels 0 .. K - 1, rows modulo 3
    C xq[3], zq[3];                // X and Z rows i .. i + 2, modulo 3
    // Row couplings, read three steps ahead and handed down the levels:
    // pjd[l] / pe[l] = the bond below / the on-site energy of row i - l
    // (0 off the grid; an open chain's last bond is 0 in the tables), so
    // that row's bond above is pjd[l + 1].
    T qjd[3], qe[3];               // rows i .. i + 2, modulo 3
    T pjd[K + 2], pe[K + 1];
    T zr[CON ? K + 1 : 1], zi[CON ? K + 1 : 1];   // zr[l]: Z row i - l (stage l of the shift register)
    C vq[CON ? K : 1][3];          // vq[l - 1][k]: v[l - 1] row i - l + k
    T rpv[CON ? K + 1 : 1], rps[CON ? K + 1 : 1];   // row parts of row i - l after level l
    double batch[8];               // three completed rows (bond, site), two zeros
    // Lane offsets of the rows a step touches, formed once per row as it
    // enters: after step i's shift ro[j] is the offset of row i + 3 - j
    // (X and Z load row i + 3, level l loads v[l - 1] row i - l + 3 and
    // stores row i - l).
    uint32_t ro[K + 4];
#pragma unroll
    for (int j = 0; j < K + 4; ++j) ro[j] = lane_off(2 - j);
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int k = 0; k < 3; ++k) yr[l][k] = yi[l][k] = T(0);
#pragma unroll
    for (int l = 0; l <= (CON ? K : 0); ++l) zr[l] = zi[l] = T(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) batch[k] = 0.0;
    // couplings of sweep step s (zero off the grid)
    auto row_jd = [&](int s) -> T {
        const int q = s_lo + s;
        if (LAY == 0 || s < 0 || s >= nsweep || (!rper && (q < 0 || q >= rows - 1))) return T(0);
        return Jr[rper ? wrapi(q, rows) : q];
    };
    auto row_e = [&](int s) -> T {
        const int q = s_lo + s;
        if (s < 0 || s >= nsweep || (!rper && (q < 0 || q >= rows))) return T(0);
        return Er[rper ? wrapi(q, rows) : q];
    };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        xq[k] = ldrow(X, k);
        if constexpr (CON) zq[k] = ldrow(Z, k);
        qjd[k] = row_jd(k);
        qe[k] = row_e(k);
    }
#pragma unroll
    for (int l = 0; l <= K + 1; ++l) pjd[l] = T(0);
#pragma unroll
    for (int l = 0; l <= K; ++l) pe[l] = T(0);
    // before step i's shift pjd[l] holds row i - 1 - l: at the start, the
    // bond above the sweep's first row (a ring, or a segment inside the grid)
    pjd[0] = (LAY != 0 && (rper || s_lo > 0)) ? Jr[rper ? wrapi(s_lo - 1, rows) : max(s_lo - 1, 0)] : T(0);
    if constexpr (CON) {
#pragma unroll
        for (int l = 0; l <= K; ++l) rpv[l] = rps[l] = T(0);
#pragma unroll
        for (int l = 1; l <= K; ++l)
#pragma unroll
            for (int k = 0; k < 3; ++k) vq[l - 1][k] = ldrow(V[l - 1], k - l);
    }
    double bond_col = 0.0, site_col = 0.0;
    const double f = tri ? 2.0 : 1.0;
    double* gV = a.gV + ((int64_t)r * a.nb + w) * a.row_stride;
    double* gR = a.gR + ((int64_t)r * a.nb + w) * a.row_stride;

    const int total = nsweep > 0 ? nsweep + K : 0;
    for (int i0 = 0; i0 < total; i0 += 3) {
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int i = i0 + u;
            // ---- level 0: row i enters (zero past the sweep)
            {
                const bool in = i < nsweep;
                const C xv = (CON && x_is_z) ? zq[u] : xq[u];
                yr[0][u] = in ? xs * xv.x : T(0);
                yi[0][u] = in ? xs * xv.y : T(0);
                if constexpr (CON) {
                    // the Z shift register advances one stage
#pragma unroll
                    for (int l = K; l >= 1; --l) {
                        zr[l] = zr[l - 1];
                        zi[l] = zi[l - 1];
                    }
                    zr[0] = zq[u].x;
                    zi[0] = zq[u].y;
                }
#pragma unroll
                for (int l = K + 1; l >= 1; --l) pjd[l] = pjd[l - 1];
#pragma unroll
                for (int l = K; l >= 1; --l) pe[l] = pe[l - 1];
                pjd[0] = qjd[u];
                pe[0] = qe[u];
#pragma unroll
                for (int j = K + 3; j >= 1; --j) ro[j] = ro[j - 1];
                ro[0] = lane_off(i + 3);
                xq[u] = load_c(X, ro[0], (C*)nullptr);
                if constexpr (CON) zq[u] = load_c(Z, ro[0], (C*)nullptr);
                qjd[u] = row_jd(i + 3);
                qe[u] = row_e(i + 3);
            }
            // ---- levels 1 .. K: row s = i - l
#pragma unroll
            for (int l = 1; l <= K; ++l) {
                const int s = i - l;
                const int su = mpos(u - l - 1, 3), sm = mpos(u - l, 3), sd = mpos(u - l + 1, 3);
                const int q = grid_row(s);
                const bool inrow = s >= 0 && s < nsweep;
                const T mr = yr[l - 1][sm], mi = yi[l - 1][sm];
                const T ur_ = yr[l - 1][su], ui_ = yi[l - 1][su];   // row s - 1
                const T dr_ = yr[l - 1][sd], di_ = yi[l - 1][sd];   // row s + 1
                const T rr = from_right(mr), ri = from_right(mi);
                const T lr = from_left(mr), li = from_left(mi);
                const bool diag = tri && cw == q;
                // neighbours below and to the left; mirrored on the stored diagonal
                const T br = diag ? rr : dr_, bi = diag ? ri : di_;
                const T ar = diag ? ur_ : lr, ai = diag ? ui_ : li;
                const bool dn = LAY != 0 && (rper || q < rows - 1);
                const T Jup = pjd[l + 1];
                const T Jdn = pjd[l];
                T d = pe[l] + ec;
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
                // Y_l = cz_l Z + s (-i)(hr + i hi) = cz_l Z + s (hi - i hr)
                const bool keep = inrow && stored(q);
                T yr_ = sg * hi, yi_ = -sg * hr;
                if constexpr (CON) {
                    const T cz = static_cast<T>(a.cz[l]);
                    yr_ = fma(cz, zr[l], yr_);
                    yi_ = fma(cz, zi[l], yi_);
                }
                yr_ = keep ? yr_ : T(0);
                yi_ = keep ? yi_ : T(0);
                if (l < K) {
                    yr[l][sm] = yr_;
                    yi[l][sm] = yi_;
                }
                const bool own = s >= o_lo && s < o_hi;
                if (!CON || l == K) store_c(yr_, yi_, Y[l - 1], (own && out) ? ro[l + 3] : kPastEnd);
                if constexpr (CON) {
                    // Im conj(u) v with u = level l's input, v = v[l - 1], per
                    // pair in the state's precision, summed in FP64
                    const C v0 = vq[l - 1][0], vp = vq[l - 1][1];
                    const T vr = from_right(v0.x), vi = from_right(v0.y);
                    const bool st = own && out && stored(q);
                    const T s0 = im_t(mr, mi, v0.x, v0.y);
                    const T hb = im_t(mr, mi, vr, vi) + im_t(rr, ri, v0.x, v0.y);
                    site_col += st ? (double)s0 : 0.0;
                    bond_col += (st && has_bond_c) ? (double)hb : 0.0;
                    const T vb = im_t(mr, mi, vp.x, vp.y) + im_t(dr_, di_, v0.x, v0.y);
                    rpv[l] += (st && dn && (!tri || cw >= q + 1)) ? vb : T(0);
                    rps[l] += (st && !diag) ? s0 : T(0);
                    // v[l - 1] advances one row
                    vq[l - 1][0] = vq[l - 1][1];
                    vq[l - 1][1] = vq[l - 1][2];
                    vq[l - 1][2] = load_c(V[l - 1], ro[l], (C*)nullptr);
                }
            }
            if constexpr (CON) {
                // row i - K is complete (stage K); the stages advance
                if (LAY != 0) {
                    batch[2 * u] = (double)rpv[K];
                    batch[2 * u + 1] = (double)rps[K];
                }
#pragma unroll
                for (int l = K; l >= 2; --l) {
                    rpv[l] = rpv[l - 1];
                    rps[l] = rps[l - 1];
                }
                rpv[1] = rps[1] = T(0);
                if (LAY != 0 && u == 2) {
                    // rows i - K - 2 .. i - K: lane 8 j ends with the wave's sum of batch[j]
                    const double t = reduce8(batch, lane);
                    const int j = lane >> 3;
                    const int s = i - K - 2 + (j >> 1);
                    if ((lane & 7) == 0 && j < 6 && s >= o_lo && s < o_hi) {
                        const int q = grid_row(s);
                        if (j & 1) gR[q] += f * t;
                        else gV[q] += f * t;
                    }
                }
            }
        }
    }
    if constexpr (CON) {
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

}  // namespace adj_pipe
}  // namespace ctqw
