// Host runtime of libctqw: the C ABI of include/ctqw.h.
//
// Stage structure of Algs. 2-3 (Sec. 3 of the paper: initialisation,
// wave-function evolution, Hamiltonian update, density-matrix
// post-processing).  Static noise: the Hamiltonian update stage is empty.
//  * initialisation  -- ctqw_plan_create / ctqw_set_params build the
//    realisation tables, Taylor orders and column bands on the host;
//    ctqw_bind uploads them once into the caller's workspace.
//  * evolution       -- ctqw_propagate launches one fused step kernel per
//    time step (all Taylor terms, Alg. 3) and a small FP64 kernel that
//    reduces the per-band norms in a fixed order and raises the alarms
//    (the "check norm" line of Alg. 3).
//  * post-processing -- the diagonal of the ensemble-averaged density matrix
//    (occupations, pair correlation), reduced in FP64 in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <complex>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/ctqw.h"
#include "ctqw_internal.hpp"
#include "adjoint_pipe.hpp"
#include "step3c.hpp"
#include "noise.hpp"
#include "density.hpp"
#include "graph.hpp"
#include "telegraph.hpp"

using namespace ctqw;

namespace {

constexpr int kMaxSites = 32768;
// Two-particle steps: batches of fewer bands than the device has SIMDs
// (256 CUs x 4) have their bands' rows split into up to kMaxRowSegments
// segments.
constexpr int kSplitTarget = 1024;
constexpr int kMaxRowSegments = 16;
thread_local std::string g_last_error;

struct Region {
    int64_t off = 0;
    int64_t bytes = 0;
};

struct Layout {
    Region reals, items, order, item_first, claim, lists, Jd, Ed, Jf, Ef, scale, norm_part,
        tail_part, norm2, tail2, status, colsum, rowsum, diag, site_off, gmembers, gfirst, gN, gout, obs, sites,
        s3, items3, M3, occ3, chunk, tbase, tsign, tstep;
    int64_t total = 0;
};

}  // namespace

struct ctqw_plan {
    ctqw_problem prob{};
    std::vector<int32_t> N;          // [R]
    std::vector<int64_t> state_off;  // [R + 1]
    std::vector<int32_t> param_off;  // [R] into the padded J / eps arrays
    int64_t param_total = 0;         // padded entries incl. the zero block
    int32_t zero_block = 0;          // offset of the all-zero row-axis block
    int32_t max_N = 0;
    int64_t site_total = 0;          // sum_r N_r
    std::vector<int64_t> site_off;   // [R]
    bool params_set = false;
    std::vector<double> J, eps, U;   // user layout (packed, unpadded)
    std::vector<double> Jpad, Epad;  // padded [param_total]
    std::vector<int32_t> order;      // [R]
    std::vector<double> xbound;      // [R] dt * Gershgorin bound of ||H_r||
    // groups (distinct N, ascending)
    std::vector<int32_t> group_N, group_first, group_members;
    std::vector<int64_t> group_out;
    int64_t obs_per_snapshot = 0;
    // work items
    std::vector<ItemDev> items;
    std::vector<Item3Dev> items3;    // three particles: plane tiles
    int k3 = 0;                      // three particles: terms per pass
    std::vector<Step3cProd> prod3;   // three particles, product form: one entry per pass
    std::vector<int32_t> item_first, item_order;
    // fused steps: runs of item_order with one Taylor order each, largest
    // order first: {order, first, end}
    std::vector<std::array<int32_t, 5>> order_runs;   // {order, first, end, paired access, two orders}
    // persistent launches: per run of order_runs, then for the whole order,
    // kClaimLists + 1 offsets of the per-XCD claim lists (relative to the
    // launch's first item)
    std::vector<int32_t> list_off;
    bool all_vec = false;            // every item takes the paired-access kernel
    bool one_depth = false;          // set while a gradient run needs one polynomial for all
    int64_t n_parts = 0;             // per-step FP64 norm partials
    int levels = 0;                  // Taylor terms per step (the batch's order)
    int chunk = 0;                   // terms per pass of a chunked step (0: fused)
    ctqw_launch launch{};
    Layout lay;
    bool tables_dirty = true;
    // binding
    bool bound = false;
    void* psi[2] = {nullptr, nullptr};
    int cur = 0;
    uint8_t* ws = nullptr;
    int64_t ws_bytes = 0;
    int64_t state_bytes_bound = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    int64_t steps_done = 0;
    bool have_step_stats = false;
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev;      // pairs (start, stop) per timed launch
    size_t ev_used = 0;              // events recorded and not yet read
    std::vector<int64_t> ev_steps;   // steps covered by each recorded pair
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
    // captured step loops: (steps, starting buffer) -> executable graph
    std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;
    // checkpointed forward run awaiting its backward pass
    void* grad_ws = nullptr;
    int64_t grad_steps = 0, grad_ckpt = 1, grad_tables = -1;
    int64_t table_version = 0;       // bumped whenever the kernel tables change
    std::string err;
    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    double tele_amp = 0.0, tele_rate = 0.0;   // switching hopping noise (0: static)
    uint64_t tele_seed = 0;
    ~ctqw_plan() {
        drop_graphs();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

namespace {

ctqw_status fail(ctqw_plan* p, ctqw_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    if (p) p->err = buf;
    return s;
}

}  // namespace

int ctqw::report_error(int status, const char* message) {
    g_last_error = message;
    return status;
}

namespace {

#define HIP_TRY(p, call)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((p), CTQW_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool is_fin(double x) { return std::isfinite(x); }

int n_bonds(const ctqw_problem& pr, int N) { return pr.boundary == CTQW_PERIODIC ? N : N - 1; }

int64_t amplitudes(const ctqw_problem& pr, int N) {
    if (pr.m == 1) return N;
    if (pr.m == 3) return (int64_t)N * N * N;
    if (pr.statistics == CTQW_BOSON || pr.statistics == CTQW_FERMION) return (int64_t)N * (N + 1) / 2;
    return (int64_t)N * N;
}

// Orders above the fused pipeline's depth run as chunked passes (one and
// two particles) or as one term per pass (three), so the cap is the user's.
constexpr int kDefaultMaxOrder = 40;
int max_order_cap(const ctqw_problem& pr) {
    return pr.taylor_max_order > 0 ? pr.taylor_max_order : kDefaultMaxOrder;
}

// a-priori remainder bound of the degree-n Taylor polynomial of exp(z),
// |z| <= x: sum_{k>n} x^k/k! <= x^(n+1)/(n+1)! / (1 - x/(n+2)).
double remainder_bound(double x, int n) {
    if (x >= n + 2) return INFINITY;
    double t = 1.0;
    for (int k = 1; k <= n + 1; ++k) t *= x / k;
    return t / (1.0 - x / (n + 2));
}

void align_region(Layout& L, Region& r, int64_t bytes) {
    L.total = (L.total + 255) & ~int64_t(255);
    r.off = L.total;
    r.bytes = bytes;
    L.total += bytes;
}

template <typename T>
T* at(ctqw_plan* p, const Region& r) {
    return reinterpret_cast<T*>(p->ws + r.off);
}

// Windows of W consecutive indices covering [0, N) with a halo of h on each
// side (the same rule as the output-aligned column bands below, without the
// row fields): {window start, first output, end of output}.  Boundaries
// inside the chain are moved down to multiples of `align` where that leaves
// an output; on an open chain the last window may run past the end.
bool bands_1d(int N, int h, int W, bool periodic, int align, std::vector<std::array<int32_t, 3>>& out) {
    if (W - 2 * h <= 0) return false;
    int lo = 0;
    while (lo < N) {
        auto aligned = [&](int c) {
            const int a = (c / align) * align;
            return a > lo ? a : c;
        };
        int w0, hi;
        if (periodic) {
            w0 = lo - h;
            const int end = w0 + W - h;
            hi = end >= N ? N : aligned(end);
        } else {
            w0 = std::max(0, lo - h);   // the last window may run past the chain's end
            hi = (w0 + W >= N) ? N : aligned(w0 + W - h);
        }
        if (hi <= lo) return false;
        out.push_back({w0, lo, hi});
        lo = hi;
    }
    return true;
}

// Terms per pass of the three-particle kernel: the launch's choice, else 3
// (complex64) or 2 (complex128), never more than the order.
int terms3(const ctqw_plan* p, int order) {
    int K = p->launch.terms_per_pass > 0 ? p->launch.terms_per_pass : (p->prob.dtype == CTQW_C128 ? 2 : 3);
    return std::max(1, std::min(K, order));
}

// Product form of the three-particle step (step3c.hpp): the roots of
// p_n(z) = sum_{k<=n} z^k / k! (Durand-Kerner iteration on n! p_n, which is
// monic, in long double, then two Newton steps), grouped into passes of at
// most K roots (conjugate pairs kept together where the sizes allow), and
// per pass c_j = e_j (-i)^j, e_j the elementary symmetric polynomials of
// -1/z_k over the pass's roots.  Fails if the passes' polynomials do not
// multiply back to p_n to 1e-13.
bool product_passes(int n, int K, std::vector<Step3cProd>& out) {
    using cl = std::complex<long double>;
    std::vector<long double> c(n + 1);   // c[k] = n! / k!
    long double f = 1.0L;
    for (int k = n; k >= 0; --k) {
        c[k] = f;
        f *= (k > 0 ? k : 1);
    }
    auto P = [&](cl z) { cl v = 0; for (int k = n; k >= 0; --k) v = v * z + c[k]; return v; };
    auto dP = [&](cl z) { cl v = 0; for (int k = n; k >= 1; --k) v = v * z + (long double)k * c[k]; return v; };
    const long double R = 1.0L + (long double)n / 2.718281828459045L;
    std::vector<cl> z(n);
    for (int k = 0; k < n; ++k) z[k] = std::polar(R, 0.4L + 6.283185307179586L * k / n);
    for (int it = 0; it < 2000; ++it) {
        long double step = 0;
        for (int k = 0; k < n; ++k) {
            cl den = 1;
            for (int j = 0; j < n; ++j)
                if (j != k) den *= z[k] - z[j];
            const cl d = P(z[k]) / den;
            z[k] -= d;
            step = std::max(step, std::abs(d));
        }
        if (step < 1e-18L) break;
    }
    for (int k = 0; k < n; ++k)
        for (int it = 0; it < 2; ++it) z[k] -= P(z[k]) / dP(z[k]);
    // order: pairs (z, conj z) by increasing real part, a real root last
    std::vector<cl> up, ordered;
    cl real_root = 0;
    bool has_real = false;
    for (const cl& r : z) {
        if (std::abs(r.imag()) < 1e-12L * std::abs(r)) { real_root = cl(r.real(), 0); has_real = true; }
        else if (r.imag() > 0) up.push_back(r);
    }
    std::sort(up.begin(), up.end(), [](const cl& a, const cl& b) { return a.real() < b.real(); });
    for (const cl& r : up) { ordered.push_back(r); ordered.push_back(std::conj(r)); }
    if (has_real) ordered.push_back(real_root);
    if ((int)ordered.size() != n) return false;
    // passes of K roots (the last takes the rest)
    out.clear();
    std::vector<cl> total(1, cl(1));
    for (int s0 = 0; s0 < n; s0 += K) {
        const int Kq = std::min(K, n - s0);
        std::vector<cl> e(Kq + 1, cl(0));
        e[0] = 1;
        for (int k = 0; k < Kq; ++k) {
            const cl w = -1.0L / ordered[s0 + k];
            for (int j = k + 1; j >= 1; --j) e[j] += w * e[j - 1];
        }
        Step3cProd pp{};
        cl rot = 1;   // (-i)^j
        for (int j = 1; j <= Kq; ++j) {
            rot *= cl(0, -1);
            const cl cj = e[j] * rot;
            pp.cre[j - 1] = (double)cj.real();
            pp.cim[j - 1] = (double)cj.imag();
        }
        pp.order = n;
        pp.k_first = std::min(K, n);
        out.push_back(pp);
        std::vector<cl> nt(total.size() + Kq, cl(0));
        for (size_t a = 0; a < total.size(); ++a)
            for (int b = 0; b <= Kq; ++b) nt[a + b] += total[a] * e[b];
        total.swap(nt);
    }
    long double inv = 1.0L;
    for (int k = 0; k <= n; ++k) {
        if (k > 0) inv /= k;
        if (std::abs(total[k] - cl(inv)) > 1e-13L * inv) return false;
    }
    return true;
}

// Column bands of one realisation for halo h (= its Taylor order) and a
// window of W columns.  A band computes its whole window and stores its
// output columns [lo, hi), which lie at least h columns inside the window
// (or at the chain's ends).  Two layouts:
//  * output-aligned (window_aligned = false): band boundaries inside the
//    chain are moved down to multiples of `align` columns where that leaves
//    the band an output column, so that the stores of neighbouring bands do
//    not share cache lines (the caller halves the alignment while it would
//    add a band); the window starts h columns before the output;
//  * window-aligned (full grids on open chains): each window starts on a
//    multiple of `align` columns, so a row of the window is read as whole
//    cache lines, and the output ends on a multiple of `out_gran` columns;
//    neighbouring bands then store parts of one line.
// On an open chain the last window is not moved back inside the chain:
// its columns past the end are lanes without data, which load nothing.
// Returns false if the halo leaves no output column.
// With `pairs` (lanes holding two adjacent columns) the window starts on an
// even column where the chain allows, so that the lanes' column pairs are
// read and written as one 16-byte access.
bool make_bands(const ctqw_problem& pr, int r, int N, int h, int W, int align, bool pairs,
                std::vector<ItemDev>& out, bool window_aligned = false, int out_gran = 1) {
    const int rows = pr.m == 1 ? 1 : N;
    const bool periodic = pr.boundary == CTQW_PERIODIC;
    const bool tri = pr.m == 2 && pr.statistics != CTQW_DISTINGUISHABLE;
    if (W - 2 * h <= 0) return false;
    window_aligned = window_aligned && !periodic && !tri && align > 1;
    int lo = 0;
    int next_w0 = 0;
    while (lo < N) {
        ItemDev it{};
        it.real = r;
        auto aligned = [&](int c) {
            const int a = (c / align) * align;
            return a > lo ? a : c;
        };
        if (window_aligned) {
            const int w0 = next_w0;   // a multiple of align, at most lo - h
            it.w0 = w0;
            it.lo = lo;
            it.hi = w0 + W >= N ? N : ((w0 + W - h) / out_gran) * out_gran;
            if (it.hi < N) next_w0 = std::max(0, ((it.hi - h) / align) * align);
        } else if (periodic) {
            int w0 = lo - h;
            if (pairs && (w0 & 1)) --w0;
            it.w0 = w0;
            it.lo = lo;
            const int end = w0 + W - h;
            it.hi = end >= N ? N : aligned(end);
        } else {
            int w0 = std::max(0, lo - h);
            if (pairs && (w0 & 1)) --w0;
            const int w1 = w0 + W;
            it.w0 = w0;
            it.lo = lo;
            it.hi = (w1 >= N) ? N : aligned(w1 - h);
        }
        if (it.hi <= it.lo) return false;
        if (periodic && rows > 1) {
            it.row0 = -h;
            it.nrows = rows + 2 * h;
        } else if (tri) {
            it.row0 = 0;
            it.nrows = std::min(rows, it.w0 + W);
        } else {
            it.row0 = 0;
            it.nrows = rows;
        }
        it.out_lo = 0;
        it.out_hi = rows;
        out.push_back(it);
        lo = it.hi;
    }
    return true;
}

ctqw_status build_tables(ctqw_plan* p) {
    const ctqw_problem& pr = p->prob;
    const int P = p->launch.cols_per_lane;
    const int W = 64 * P;
    int maxn = 0;
    for (int64_t r = 0; r < pr.R; ++r) maxn = std::max(maxn, p->order[r]);
    const int dtype = pr.dtype == CTQW_C128 ? 1 : 0;
    const int fused = pr.m == 3 ? maxn : step_levels_bucket(dtype, P, maxn);
    // chunked passes when the order has no fused pipeline, or on request
    const int chunk = (pr.m != 3 && (fused < 0 || p->launch.chunked)) ? chunk_depth(dtype) : 0;
    const int levels = maxn;
    const int band_W = chunk ? 64 : W;          // chunked passes run one column per lane
    const int halo = chunk ? chunk : levels;
    const int amp_bytes = dtype ? 16 : 8;
    const int align = std::max(1, p->launch.band_align / amp_bytes);
    std::vector<ItemDev> items;
    std::vector<int32_t> first(pr.R + 1, 0);
    int64_t n_parts = 0;
    std::vector<Item3Dev> items3;
    int k3 = 0;
    if (pr.m == 3) {
        // tiles of the (x2, x3) plane swept over x1, halo = terms per pass;
        // one norm partial per tile
        k3 = terms3(p, maxn);
        p->prod3.clear();
        if (p->launch.three_form == 1 && maxn > k3 && !product_passes(maxn, k3, p->prod3))
            return fail(p, CTQW_ERR_UNSUPPORTED, "no product form of the order-%d Taylor polynomial", maxn);
        const int rows = step3c_rows_per_block(dtype, k3);
        if (rows <= 0) return fail(p, CTQW_ERR_UNSUPPORTED, "%d terms per pass are not compiled", k3);
        const bool periodic = pr.boundary == CTQW_PERIODIC;
        for (int64_t r = 0; r < pr.R; ++r) {
            const int N = p->N[r];
            std::vector<std::array<int32_t, 3>> yb, zb, trial;
            if (!bands_1d(N, k3, rows, periodic, 1, yb) || !bands_1d(N, k3, 64, periodic, 1, zb))
                return fail(p, CTQW_ERR_UNSUPPORTED, "%d terms per pass leave a tile no output", k3);
            // x3 band boundaries on whole cache lines where that adds no band
            for (int a = std::max(1, p->launch.band_align / amp_bytes); a > 1; a /= 2) {
                trial.clear();
                if (bands_1d(N, k3, 64, periodic, a, trial) && trial.size() <= zb.size()) {
                    zb.swap(trial);
                    break;
                }
            }
            first[r] = (int32_t)items3.size();
            for (const auto& y : yb)
                for (const auto& zz : zb) {
                    Item3Dev t{};
                    t.real = (int32_t)r;
                    t.z0 = zz[0];
                    t.zlo = zz[1];
                    t.zhi = zz[2];
                    t.y0 = y[0];
                    t.ylo = y[1];
                    t.yhi = y[2];
                    t.x0 = periodic ? -k3 : 0;
                    t.nplanes = periodic ? N + 2 * k3 : N;
                    t.plane_lo = 0;
                    t.plane_hi = N;
                    items3.push_back(t);
                }
            if (items3.size() > (size_t)INT32_MAX) return fail(p, CTQW_ERR_OUT_OF_MEMORY, "too many tiles");
        }
        first[pr.R] = (int32_t)items3.size();
        n_parts = (int64_t)items3.size();
    } else {
        for (int64_t r = 0; r < pr.R; ++r) {
            first[r] = (int32_t)items.size();
            // the largest alignment (at most the requested one) that needs no
            // more bands than unaligned boundaries
            const bool pairs_r = band_W == 128 && dtype == 0;
            std::vector<ItemDev> plain, trial;
            if (!make_bands(pr, (int)r, p->N[r], halo, band_W, 1, pairs_r, plain))
                return fail(p, CTQW_ERR_UNSUPPORTED, "Taylor order %d too deep for a %d-column band", halo, band_W);
            const std::vector<ItemDev>* use = &plain;
            if (p->launch.band_mode == 1 && align > 1) {
                // window-aligned bands; outputs end on 32-byte boundaries
                const int gran = std::max(1, std::min(align, 32 / amp_bytes));
                if (make_bands(pr, (int)r, p->N[r], halo, band_W, align, pairs_r, trial, true, gran) &&
                    trial.size() <= plain.size() + 1)
                    use = &trial;
            } else {
                for (int a = align; a > 1; a /= 2) {
                    trial.clear();
                    if (make_bands(pr, (int)r, p->N[r], halo, band_W, a, pairs_r, trial) &&
                        trial.size() <= plain.size()) {
                        use = &trial;
                        break;
                    }
                }
            }
            items.insert(items.end(), use->begin(), use->end());
        }
        // Few bands: a band's rows are swept in order by one wave, so the
        // step lasts as long as the longest sweep.  Split each band's output
        // rows into segments, each swept from `halo` rows before its first
        // output row to `halo` rows after its last (the rows the pipeline
        // needs to bring its deepest term up to date).
        const int seg_cap = p->launch.row_segments == 0
                                ? ((int64_t)items.size() < kSplitTarget ? kMaxRowSegments : 1)
                                : p->launch.row_segments;
        if (!chunk && pr.m == 2 && seg_cap > 1) {
            const bool periodic = pr.boundary == CTQW_PERIODIC;
            const int64_t want = p->launch.row_segments == 0
                                     ? (kSplitTarget + (int64_t)items.size() - 1) / (int64_t)items.size()
                                     : seg_cap;
            const int S = (int)std::min<int64_t>(seg_cap, want);
            std::vector<ItemDev> split;
            split.reserve(items.size() * S);
            size_t k = 0;
            for (int64_t r = 0; r < pr.R; ++r) {
                first[r] = (int32_t)split.size();
                for (; k < items.size() && items[k].real == r; ++k) {
                    const ItemDev& it = items[k];
                    const int e_lo = std::max(it.out_lo, it.row0);
                    const int e_hi = std::min(it.out_hi, it.row0 + it.nrows);
                    const int s = std::min(S, (e_hi - e_lo) / std::max(8, 2 * halo));
                    if (s <= 1) {
                        split.push_back(it);
                        continue;
                    }
                    for (int q = 0; q < s; ++q) {
                        ItemDev t = it;
                        t.out_lo = e_lo + (int)((int64_t)(e_hi - e_lo) * q / s);
                        t.out_hi = e_lo + (int)((int64_t)(e_hi - e_lo) * (q + 1) / s);
                        t.row0 = periodic ? t.out_lo - halo : std::max(it.row0, t.out_lo - halo);
                        const int stop = periodic ? t.out_hi + halo : std::min(it.row0 + it.nrows, t.out_hi + halo);
                        t.nrows = stop - t.row0;
                        split.push_back(t);
                    }
                }
            }
            items.swap(split);
        }
        first[pr.R] = (int32_t)items.size();
        n_parts = (int64_t)items.size();
    }
    if (items.size() > (size_t)INT32_MAX) return fail(p, CTQW_ERR_OUT_OF_MEMORY, "too many work items");
    // Fused steps run each realisation at its own a-priori order: the items
    // are ordered by order (largest first), then by kernel variant, then by
    // cost, and each run of one (order, variant) is a launch of that depth.
    // Paired 16-byte access (complex64, two columns per lane, full grid)
    // needs an even chain length and an even window start and output range.
    const bool pairs = !chunk && P == 2 && dtype == 0 && !(pr.m == 2 && pr.statistics != CTQW_DISTINGUISHABLE);
    std::vector<int32_t> ord(items.size());
    std::vector<int64_t> cost(items.size());
    std::vector<int32_t> iord(items.size()), ivec(items.size());
    bool all_vec = !items.empty();
    for (size_t k = 0; k < items.size(); ++k) {
        const ItemDev& it = items[k];
        ord[k] = (int32_t)k;
        cost[k] = (int64_t)(it.nrows + halo);
        iord[k] = chunk ? levels : p->order[it.real];
        ivec[k] = (pairs && (p->N[it.real] & 1) == 0 && (it.w0 & 1) == 0 && (it.lo & 1) == 0 && (it.hi & 1) == 0)
                      ? 1 : 0;
        all_vec = all_vec && ivec[k];
    }
    // Complex64 full-grid launches take two adjacent orders n, n - 1 together
    // (kernel variant TWO): their items are mixed largest first, so the
    // instruction-heavier and the lighter items share the device.
    std::vector<int32_t> igrp(items.size());
    {
        // (measured: a gain at two columns per lane, a loss at one)
        const bool two_ok =
            !chunk && dtype == 0 && P == 2 && !(pr.m == 2 && pr.statistics != CTQW_DISTINGUISHABLE) && pr.m != 3;
        std::vector<int32_t> present;
        for (size_t k = 0; k < items.size(); ++k) present.push_back(iord[k]);
        std::sort(present.begin(), present.end(), std::greater<int32_t>());
        present.erase(std::unique(present.begin(), present.end()), present.end());
        std::map<int32_t, int32_t> group_of;
        for (size_t q = 0; q < present.size(); ++q) {
            group_of[present[q]] = present[q];
            if (two_ok && q + 1 < present.size() && present[q + 1] == present[q] - 1) {
                group_of[present[q + 1]] = present[q];
                ++q;
            }
        }
        for (size_t k = 0; k < items.size(); ++k) igrp[k] = group_of[iord[k]];
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
        if (igrp[a] != igrp[b]) return igrp[a] > igrp[b];
        if (ivec[a] != ivec[b]) return ivec[a] > ivec[b];
        return cost[a] > cost[b];
    });
    p->order_runs.clear();
    for (size_t k = 0; k < ord.size(); ++k) {
        const int32_t g = igrp[ord[k]], v = ivec[ord[k]], two = iord[ord[k]] != g;
        if (p->order_runs.empty() || p->order_runs.back()[0] != g || p->order_runs.back()[3] != v)
            p->order_runs.push_back({g, (int32_t)k, (int32_t)k, v, 0});
        p->order_runs.back()[2] = (int32_t)k + 1;
        if (two) p->order_runs.back()[4] = 1;
    }
    // Persistent launches: split each run into one claim list per XCD.
    // Consecutive items of one realisation (its adjacent bands, which share
    // halo columns) go to one list as a cluster; clusters are dealt out in
    // the processing order (largest first) to the list with the least work
    // so far, and each list keeps that order.
    {
        const int XL = kClaimLists;
        p->list_off.assign((p->order_runs.size() + 1) * (XL + 1), 0);
        auto split_range = [&](int32_t k0, int32_t k1, int32_t* off) {
            const int32_t n = k1 - k0;
            if (!p->launch.persistent || n <= 0) {
                off[0] = 0;
                for (int x = 1; x <= XL; ++x) off[x] = n;
                return;
            }
            std::vector<std::vector<int32_t>> lists(XL);
            std::vector<int64_t> load(XL, 0);
            for (int32_t k = k0; k < k1;) {
                const int32_t real = items[ord[k]].real;
                int32_t e = k;
                int64_t c = 0;
                while (e < k1 && items[ord[e]].real == real) c += cost[ord[e++]];
                const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                for (int32_t q = k; q < e; ++q) lists[x].push_back(ord[q]);
                load[x] += c;
                k = e;
            }
            int32_t at_ = 0;
            off[0] = 0;
            for (int x = 0; x < XL; ++x) {
                std::copy(lists[x].begin(), lists[x].end(), ord.begin() + k0 + at_);
                at_ += (int32_t)lists[x].size();
                off[x + 1] = at_;
            }
        };
        for (size_t q = 0; q < p->order_runs.size(); ++q)
            split_range(p->order_runs[q][1], p->order_runs[q][2], &p->list_off[q * (XL + 1)]);
        // whole order (launches at one depth): the runs' lists when there is
        // one run, else one list
        int32_t* whole = &p->list_off[p->order_runs.size() * (XL + 1)];
        if (p->order_runs.size() == 1) {
            std::copy(p->list_off.begin(), p->list_off.begin() + (XL + 1), whole);
        } else {
            whole[0] = 0;
            for (int x = 1; x <= XL; ++x) whole[x] = (int32_t)ord.size();
        }
    }
    p->all_vec = all_vec;
    p->items3.swap(items3);
    p->k3 = k3;
    p->items.swap(items);
    p->item_first.swap(first);
    p->item_order.swap(ord);
    p->levels = levels;
    p->chunk = chunk;

    // workspace layout
    Layout L;
    const int64_t R = pr.R;
    const int64_t nit = (int64_t)p->items.size();
    const int64_t G = (int64_t)p->group_N.size();
    align_region(L, L.reals, R * (int64_t)sizeof(RealDev));
    align_region(L, L.items, nit * (int64_t)sizeof(ItemDev));
    align_region(L, L.order, nit * 4);
    align_region(L, L.item_first, (R + 1) * 4);
    align_region(L, L.claim, 4 * kClaimLists);   // persistent launch: claim counters
    align_region(L, L.lists, (int64_t)p->list_off.size() * 4);
    align_region(L, L.Jd, p->param_total * 8);
    align_region(L, L.Ed, p->param_total * 8);
    align_region(L, L.Jf, p->param_total * 4);
    align_region(L, L.Ef, p->param_total * 4);
    align_region(L, L.scale, R * 8);
    align_region(L, L.norm_part, n_parts * 8);
    align_region(L, L.tail_part, n_parts * 8);
    align_region(L, L.norm2, R * 8);
    align_region(L, L.tail2, R * 8);
    align_region(L, L.status, 16);
    align_region(L, L.colsum, p->site_total * 8);
    align_region(L, L.rowsum, p->site_total * 8);
    align_region(L, L.diag, p->site_total * 8);
    align_region(L, L.site_off, R * 8);
    align_region(L, L.gmembers, R * 4);
    align_region(L, L.gfirst, (G + 1) * 4);
    align_region(L, L.gN, G * 4);
    align_region(L, L.gout, G * 8);
    align_region(L, L.obs, p->obs_per_snapshot * 8);
    align_region(L, L.sites, R * pr.m * 4);
    if (pr.m == 3) {
        // tiles, pass buffers (the partial sum and two for the last term of
        // a pass, used alternately) and the two-body marginals
        const int64_t sb = p->state_off.back() * (pr.dtype == CTQW_C128 ? 16 : 8);
        const int64_t NN = (int64_t)p->max_N * p->max_N;
        align_region(L, L.items3, (int64_t)p->items3.size() * (int64_t)sizeof(Item3Dev));
        align_region(L, L.s3, 3 * ((sb + 255) & ~int64_t(255)));
        align_region(L, L.M3, R * 3 * NN * 8);
        align_region(L, L.occ3, G * NN * 8);
    }
    if (p->tele_amp > 0.0) {
        // switching noise: baseline hoppings, current signs, step counter
        align_region(L, L.tbase, p->param_total * 8);
        align_region(L, L.tsign, p->param_total * 4);
        align_region(L, L.tstep, 16);
    }
    if (chunk) {
        // two buffers for the last term of a pass, one for the partial sum
        const int64_t sb = p->state_off.back() * (pr.dtype == CTQW_C128 ? 16 : 8);
        align_region(L, L.chunk, 3 * ((sb + 255) & ~int64_t(255)));
    }
    L.total = (L.total + 255) & ~int64_t(255);
    p->n_parts = n_parts;
    p->lay = L;
    p->tables_dirty = true;
    p->drop_graphs();
    ++p->table_version;
    return CTQW_OK;
}

ctqw_status upload_tables(ctqw_plan* p) {
    const ctqw_problem& pr = p->prob;
    const Layout& L = p->lay;
    const int64_t R = pr.R;
    std::vector<RealDev> reals(R);
    for (int64_t r = 0; r < R; ++r) {
        RealDev& d = reals[r];
        d.state_off = p->state_off[r];
        d.N = p->N[r];
        // grid rows of N amplitudes: 1 (one particle), N (two), N^2 (three)
        d.rows = pr.m == 1 ? 1 : (pr.m == 3 ? p->N[r] * p->N[r] : p->N[r]);
        // Fused two-dimensional steps run the realisation's own order;
        // one-depth launches (chunked passes, gradients, three particles)
        // run the batch's largest.
        const int n = (p->chunk || pr.m == 3) ? p->levels : p->order[r];
        const int nmax = p->levels;
        const double x = p->xbound[r];
        d.order = n;
        d.param_off = p->param_off[r];
        d.row_param_off = pr.m == 1 ? p->zero_block : p->param_off[r];
        d.flags = (pr.boundary == CTQW_PERIODIC ? RF_PERIODIC : 0) |
                  (pr.m == 2 && pr.statistics != CTQW_DISTINGUISHABLE ? RF_TRIANGLE : 0) |
                  (pr.m == 2 && pr.statistics == CTQW_FERMION ? RF_FERMION : 0) |
                  (pr.interaction == CTQW_INT_NEAREST ? RF_NEAREST : 0);
        {
            // no on-site energies: the diagonal of H is the interaction alone
            bool zero = true;
            for (int i = 0; i < p->N[r] && zero; ++i) zero = p->Epad[p->param_off[r] + i] == 0.0;
            if (zero) d.flags |= RF_NO_EPS;
        }
        d.U = pr.m == 1 ? 0.0 : p->U[r];
        // remainder estimate: ||sum_{j>n} Phi^(j)|| <= ||Phi^(n)|| (x/(n+1)) / (1 - x/(n+2))
        d.tail_factor = (x < n + 2) ? (x / (n + 1)) / (1.0 - x / (n + 2)) : INFINITY;
        d.tail_factor_max = (x < nmax + 2) ? (x / (nmax + 1)) / (1.0 - x / (nmax + 2)) : INFINITY;
    }
    // Step kernels read J and eps pre-multiplied by dt.
    const double dt = pr.dt;
    std::vector<double> Jd(p->Jpad.size()), Ed(p->Epad.size());
    for (size_t k = 0; k < Jd.size(); ++k) {
        Jd[k] = dt * p->Jpad[k];
        Ed[k] = dt * p->Epad[k];
    }
    std::vector<float> tsign;
    if (p->tele_amp > 0.0) {
        // switching noise: initial signs (draw s = -1), J = Jbar + a * sign
        tsign.assign(p->Jpad.size(), 0.0f);
        const uint32_t key[2] = {(uint32_t)(p->tele_seed & 0xffffffffu) ^ 0x54454C45u, (uint32_t)(p->tele_seed >> 32)};
        for (int64_t r = 0; r < R; ++r) {
            const int nb = n_bonds(pr, p->N[r]);
            for (int i = 0; i < nb; ++i) {
                const uint32_t ctr[4] = {(uint32_t)i, 0u, (uint32_t)((uint64_t)r & 0xffffffffu), (uint32_t)((uint64_t)r >> 32)};
                uint32_t w[4];
                philox4x32_10(ctr, key, w);
                const int64_t k = p->param_off[r] + i;
                tsign[k] = unit_double(w[0], w[1]) < 0.5 ? 1.0f : -1.0f;
                Jd[k] = dt * (p->Jpad[k] + p->tele_amp * (double)tsign[k]);
            }
        }
    }
    std::vector<float> Jf(Jd.begin(), Jd.end()), Ef(Ed.begin(), Ed.end());
    std::vector<double> ones(R, 1.0);
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;
    hipStream_t s = p->stream;
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.reals.off, reals.data(), L.reals.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.items.off, p->items.data(), L.items.bytes, h2d, s));
    if (L.items3.bytes > 0)
        HIP_TRY(p, hipMemcpyAsync(p->ws + L.items3.off, p->items3.data(), L.items3.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.order.off, p->item_order.data(), L.order.bytes, h2d, s));
    if (L.lists.bytes > 0)
        HIP_TRY(p, hipMemcpyAsync(p->ws + L.lists.off, p->list_off.data(), L.lists.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.item_first.off, p->item_first.data(), L.item_first.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.Jd.off, Jd.data(), L.Jd.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.Ed.off, Ed.data(), L.Ed.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.Jf.off, Jf.data(), L.Jf.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.Ef.off, Ef.data(), L.Ef.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.scale.off, ones.data(), L.scale.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.site_off.off, p->site_off.data(), L.site_off.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.gmembers.off, p->group_members.data(), L.gmembers.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.gfirst.off, p->group_first.data(), L.gfirst.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.gN.off, p->group_N.data(), L.gN.bytes, h2d, s));
    HIP_TRY(p, hipMemcpyAsync(p->ws + L.gout.off, p->group_out.data(), L.gout.bytes, h2d, s));
    HIP_TRY(p, launch_fill_zero(p->ws + L.status.off, 32, s));
    if (p->tele_amp > 0.0) {
        HIP_TRY(p, hipMemcpyAsync(p->ws + L.tbase.off, p->Jpad.data(), L.tbase.bytes, h2d, s));
        HIP_TRY(p, hipMemcpyAsync(p->ws + L.tsign.off, tsign.data(), L.tsign.bytes, h2d, s));
        HIP_TRY(p, launch_fill_zero(p->ws + L.tstep.off, 16, s));
    }
    HIP_TRY(p, hipStreamSynchronize(s));
    p->tables_dirty = false;
    return CTQW_OK;
}

ctqw_status ensure_ready(ctqw_plan* p) {
    if (!p->bound) return fail(p, CTQW_ERR_STATE, "plan is not bound to device memory");
    if (p->lay.total > p->ws_bytes)
        return fail(p, CTQW_ERR_STATE, "workspace too small (%lld < %lld bytes); query ctqw_sizes and re-bind",
                    (long long)p->ws_bytes, (long long)p->lay.total);
    if (p->tables_dirty) return upload_tables(p);
    return CTQW_OK;
}

StepConfig step_config(ctqw_plan* p) {
    StepConfig c{};
    c.dtype = p->prob.dtype == CTQW_C128 ? 1 : 0;
    c.kahan = (c.dtype == 0 && p->prob.accumulation == CTQW_ACC_KAHAN) ? 1 : 0;
    c.triangle = (p->prob.m == 2 && p->prob.statistics != CTQW_DISTINGUISHABLE) ? 1 : 0;
    c.cols_per_lane = p->chunk ? 1 : p->launch.cols_per_lane;
    c.levels = p->chunk ? p->chunk : p->levels;
    c.waves_per_block = p->launch.waves_per_block;
    c.persistent = p->launch.persistent;
    c.grid_blocks = 0;
    return c;
}

// Grid of one step launch over `n_items` items (regular: one wave per item;
// persistent: the device's resident waves, at most the items' blocks).
ctqw_status grid_for(ctqw_plan* p, StepConfig& c, int* n_waves, int64_t n_items = -1) {
    if (n_items < 0) n_items = (int64_t)p->items.size();
    int max_threads = 0;
    if (p->chunk) HIP_TRY(p, chunk_max_block(c, &max_threads));
    else HIP_TRY(p, step_max_block(c, &max_threads));
    if (64 * c.waves_per_block > max_threads)
        return fail(p, CTQW_ERR_UNSUPPORTED, "%d waves per block exceed this kernel's %d threads", c.waves_per_block,
                    max_threads);
    if (!c.persistent) {
        *n_waves = (int)n_items;
        return CTQW_OK;
    }
    // one claim per group plus one final claim per block in an int32 counter
    if (n_items >= (int64_t(1) << 30))
        return fail(p, CTQW_ERR_UNSUPPORTED, "persistent launch takes at most 2^30 work items per step");
    int per_cu = 0;
    if (p->chunk) HIP_TRY(p, chunk_occupancy(c, &per_cu));
    else HIP_TRY(p, step_occupancy(c, &per_cu));
    if (p->launch.waves_per_cu > 0) per_cu = std::max(1, p->launch.waves_per_cu / c.waves_per_block);
    if (per_cu < 1) per_cu = 1;
    int64_t blocks = (int64_t)p->cu_count * per_cu;
    const int64_t need = (n_items + c.waves_per_block - 1) / c.waves_per_block;
    blocks = std::max<int64_t>(1, std::min(blocks, need));
    c.grid_blocks = (int)blocks;
    *n_waves = (int)(blocks * c.waves_per_block);
    return CTQW_OK;
}

// Timing: an event pair around each step kernel (eager) or around each
// replay of a captured step loop, which then counts for its `steps` steps.
ctqw_status record_event(ctqw_plan* p, int which, int64_t steps = 1) {
    if (which == 0 && p->ev_used + 2 > p->ev.size()) {
        for (int k = 0; k < 2; ++k) {
            hipEvent_t e;
            HIP_TRY(p, hipEventCreate(&e));
            p->ev.push_back(e);
        }
    }
    HIP_TRY(p, hipEventRecord(p->ev[p->ev_used + which], p->stream));
    if (which == 1) {
        p->ev_steps.resize(p->ev_used / 2 + 1);
        p->ev_steps[p->ev_used / 2] = steps;
        p->ev_used += 2;
    }
    return CTQW_OK;
}

ctqw_status enqueue_finalize(ctqw_plan* p) {
    const Layout& L = p->lay;
    FinalizeArgs f{};
    f.item_first = at<int32_t>(p, L.item_first);
    f.norm_part = at<double>(p, L.norm_part);
    f.tail_part = at<double>(p, L.tail_part);
    f.reals = at<RealDev>(p, L.reals);
    f.norm2 = at<double>(p, L.norm2);
    f.tail2 = at<double>(p, L.tail2);
    f.scale = at<double>(p, L.scale);
    f.status = at<int32_t>(p, L.status);
    f.R = p->prob.R;
    f.tol2 = p->prob.taylor_tol > 0 ? p->prob.taylor_tol * p->prob.taylor_tol : 0.0;
    f.norm_alarm = p->prob.norm_alarm;
    f.renormalize = p->prob.renormalize;
    f.use_max = (p->chunk || p->one_depth) ? 1 : 0;
    HIP_TRY(p, launch_finalize(f, p->stream));
    return CTQW_OK;
}

// Three particles: ceil(n / K) passes of the chained kernel from psi[cur]
// into psi[1-cur].  Pass q continues the series from the last term of pass
// q-1 (two workspace buffers, alternately) and the partial sum, which
// alternates between the workspace and the output so that the last pass
// writes the output and no pass updates its own input; the last pass takes
// the remaining n - qK terms.
ctqw_status enqueue_telegraph(ctqw_plan* p);

ctqw_status enqueue_step3(ctqw_plan* p) {
    {
        const ctqw_status st = enqueue_telegraph(p);
        if (st != CTQW_OK) return st;
    }
    const Layout& L = p->lay;
    const ctqw_problem& pr = p->prob;
    const int dtype = pr.dtype == CTQW_C128 ? 1 : 0;
    const int64_t sb = (p->state_off.back() * (dtype ? 16 : 8) + 255) & ~int64_t(255);
    uint8_t* s3 = p->ws + L.s3.off;
    uint8_t* acc_tmp = s3;
    uint8_t* seed_buf[2] = {s3 + sb, s3 + 2 * sb};
    const void* in = p->psi[p->cur];
    void* out = p->psi[1 - p->cur];
    const int n = p->levels, K = p->k3;
    const int passes = (n + K - 1) / K;
    auto acc_buf = [&](int q) -> void* { return ((passes - 1 - q) & 1) == 0 ? out : static_cast<void*>(acc_tmp); };
    auto inv_fact = [](int k) {
        double prod = 1.0;
        for (int i = 2; i <= k; ++i) prod *= i;
        return 1.0 / prod;
    };
    Step3cArgs a{};
    a.reals = at<RealDev>(p, L.reals);
    a.items = at<Item3Dev>(p, L.items3);
    a.Jt = dtype ? static_cast<const void*>(at<double>(p, L.Jd)) : static_cast<const void*>(at<float>(p, L.Jf));
    a.Et = dtype ? static_cast<const void*>(at<double>(p, L.Ed)) : static_cast<const void*>(at<float>(p, L.Ef));
    a.scale = at<double>(p, L.scale);
    a.norm_part = at<double>(p, L.norm_part);
    a.tail_part = at<double>(p, L.tail_part);
    a.dt = pr.dt;
    a.n_items = (int32_t)p->items3.size();
    a.tail_coef = inv_fact(n);
    ctqw_status st;
    if (p->timing && (st = record_event(p, 0)) != CTQW_OK) return st;
    if (!p->prod3.empty() && passes > 1) {
        // product form: pass q maps its input to q_q(z) input; the passes
        // alternate between two buffers and the last writes the new state
        void* tmp[2] = {acc_tmp, seed_buf[0]};
        const void* x = in;
        for (int q = 0; q < passes; ++q) {
            const int Kq = std::min(K, n - q * K);
            a.x_in = x;
            a.base_in = x;
            a.sum_out = q == passes - 1 ? out : tmp[q & 1];
            a.seed_out = nullptr;
            for (int j = 0; j < 4; ++j) a.coef[j] = 0.0;
            a.first = q == 0;
            a.last = q == passes - 1;
            a.tail_level = 0;
            HIP_TRY(p, launch_step3c_prod(a, p->prod3[q], dtype, Kq, p->stream));
            x = a.sum_out;
        }
    } else
    for (int q = 0; q < passes; ++q) {
        const int s0 = q * K;
        const int Kq = std::min(K, n - s0);
        a.x_in = q == 0 ? in : seed_buf[(q - 1) & 1];
        a.base_in = q == 0 ? in : acc_buf(q - 1);
        a.sum_out = acc_buf(q);
        a.seed_out = q == passes - 1 ? nullptr : seed_buf[q & 1];
        for (int j = 0; j < 4; ++j) a.coef[j] = j < Kq ? inv_fact(s0 + j + 1) : 0.0;
        a.first = q == 0;
        a.last = q == passes - 1;
        a.tail_level = a.last ? Kq : 0;
        HIP_TRY(p, launch_step3c(a, dtype, Kq, p->stream));
    }
    if (p->timing && (st = record_event(p, 1)) != CTQW_OK) return st;
    if ((st = enqueue_finalize(p)) != CTQW_OK) return st;
    p->cur = 1 - p->cur;
    p->steps_done += 1;
    p->have_step_stats = true;
    return CTQW_OK;
}

// The step kernel(s) from `in` to `out`: one fused launch, or the passes of
// a chunked step.  Pass q of Q continues the series from the last term of
// pass q-1 (two workspace buffers, alternately) and the partial sum, which
// alternates between the workspace and `out` so that the last pass writes
// `out` and no pass updates its own input.
ctqw_status enqueue_step_kernels(ctqw_plan* p, const void* in, void* out) {
    const Layout& L = p->lay;
    StepConfig c = step_config(p);
    c.vec = (!p->chunk && p->all_vec) ? 1 : 0;
    int n_waves = 0;
    ctqw_status st = grid_for(p, c, &n_waves);
    if (st != CTQW_OK) return st;
    StepArgs a{};
    a.psi_in = in;
    a.psi_out = out;
    a.reals = at<RealDev>(p, L.reals);
    a.items = at<ItemDev>(p, L.items);
    a.item_order = at<int32_t>(p, L.order);
    a.claim = at<int32_t>(p, L.claim);
    a.list_off = at<int32_t>(p, L.lists) + p->order_runs.size() * (kClaimLists + 1);   // whole order
    a.n_items = (int32_t)p->items.size();
    a.n_waves = n_waves;
    a.Jd = at<double>(p, L.Jd);
    a.Ed = at<double>(p, L.Ed);
    a.Jf = at<float>(p, L.Jf);
    a.Ef = at<float>(p, L.Ef);
    a.scale = at<double>(p, L.scale);
    a.norm_part = at<double>(p, L.norm_part);
    a.tail_part = at<double>(p, L.tail_part);
    a.dt = p->prob.dt;
    a.persistent = c.persistent;
    if (!p->chunk) {
        if (p->one_depth || p->order_runs.empty()) {
            // one launch at the batch's largest order for every item
            // (paired access only when every item allows it)
            if (c.persistent) HIP_TRY(p, launch_fill_zero(a.claim, 4 * kClaimLists, p->stream));
            HIP_TRY(p, launch_step(c, a, p->stream));
            return CTQW_OK;
        }
        // one launch per run of items (one order, or two adjacent orders),
        // each item at its own depth
        const int32_t* order_base = at<int32_t>(p, L.order);
        const int32_t* lists_base = at<int32_t>(p, L.lists);
        for (size_t q = 0; q < p->order_runs.size(); ++q) {
            const auto& run = p->order_runs[q];
            StepConfig cr = step_config(p);
            cr.levels = run[0];
            cr.vec = run[3];
            cr.two = run[4];
            const int64_t n = run[2] - run[1];
            if ((st = grid_for(p, cr, &n_waves, n)) != CTQW_OK) return st;
            a.item_order = order_base + run[1];
            a.list_off = lists_base + q * (kClaimLists + 1);
            a.n_items = (int32_t)n;
            a.n_waves = n_waves;
            if (cr.persistent) HIP_TRY(p, launch_fill_zero(a.claim, 4 * kClaimLists, p->stream));
            HIP_TRY(p, launch_step(cr, a, p->stream));
        }
        return CTQW_OK;
    }
    const int n = p->levels, K = p->chunk;
    const int passes = (n + K - 1) / K;
    const int64_t sb = (p->state_off.back() * (c.dtype ? 16 : 8) + 255) & ~int64_t(255);
    uint8_t* seed_buf[2] = {p->ws + L.chunk.off, p->ws + L.chunk.off + sb};
    uint8_t* acc_tmp = p->ws + L.chunk.off + 2 * sb;
    auto acc_buf = [&](int q) -> void* { return ((passes - 1 - q) & 1) == 0 ? out : acc_tmp; };
    // 1/k! as one division of the product, as the fused kernel's constants
    auto inv_fact = [](int k) {
        double prod = 1.0;
        for (int i = 2; i <= k; ++i) prod *= i;
        return 1.0 / prod;
    };
    const double inv_fact_n = inv_fact(n);
    for (int q = 0; q < passes; ++q) {
        const int s0 = q * K;
        a.psi_in = q == 0 ? in : seed_buf[(q - 1) & 1];
        a.acc_in = q == 0 ? in : acc_buf(q - 1);
        a.psi_out = acc_buf(q);
        a.seed_out = q == passes - 1 ? nullptr : seed_buf[q & 1];
        for (int j = 1; j <= 16; ++j) a.coef[j - 1] = (j <= K && s0 + j <= n) ? inv_fact(s0 + j) : 0.0;
        a.first = q == 0;
        a.last = q == passes - 1;
        a.tail_level = a.last ? n - s0 : 0;
        a.tail_coef = inv_fact_n;
        if (c.persistent) HIP_TRY(p, launch_fill_zero(a.claim, 4 * kClaimLists, p->stream));
        HIP_TRY(p, launch_chunk_pass(c, a, p->stream));
    }
    return CTQW_OK;
}

// Switching noise: flip the bonds' signs for this step and rewrite the
// dt-scaled hopping tables (before the step's kernels).
ctqw_status enqueue_telegraph(ctqw_plan* p) {
    if (p->tele_amp <= 0.0) return CTQW_OK;
    const Layout& L = p->lay;
    TeleArgs t{};
    t.reals = at<RealDev>(p, L.reals);
    t.Jbase = at<double>(p, L.tbase);
    t.sign = at<float>(p, L.tsign);
    t.step = at<int32_t>(p, L.tstep);
    t.Jd = at<double>(p, L.Jd);
    t.Jf = at<float>(p, L.Jf);
    t.dt = p->prob.dt;
    t.amp = p->tele_amp;
    t.p_flip = -std::expm1(-p->tele_rate * p->prob.dt);
    t.key0 = (uint32_t)(p->tele_seed & 0xffffffffu) ^ 0x54454C45u;
    t.key1 = (uint32_t)(p->tele_seed >> 32);
    t.R = p->prob.R;
    HIP_TRY(p, launch_telegraph(t, p->max_N, p->stream));
    return CTQW_OK;
}

ctqw_status enqueue_step(ctqw_plan* p) {
    if (p->prob.m == 3) return enqueue_step3(p);
    ctqw_status st;
    if ((st = enqueue_telegraph(p)) != CTQW_OK) return st;
    if (p->timing && (st = record_event(p, 0)) != CTQW_OK) return st;
    if ((st = enqueue_step_kernels(p, p->psi[p->cur], p->psi[1 - p->cur])) != CTQW_OK) return st;
    if (p->timing && (st = record_event(p, 1)) != CTQW_OK) return st;
    if ((st = enqueue_finalize(p)) != CTQW_OK) return st;
    p->cur = 1 - p->cur;
    p->steps_done += 1;
    p->have_step_stats = true;
    return CTQW_OK;
}

// One step kernel from `in` to `out` (no monitoring), for the adjoint's
// recomputation: every realisation at the batch's largest order.
ctqw_status enqueue_step_io(ctqw_plan* p, const void* in, void* out) {
    if (p->prob.m == 3) return fail(p, CTQW_ERR_UNSUPPORTED, "recomputation is built for one and two particles");
    const bool was = p->one_depth;
    p->one_depth = true;
    const ctqw_status st = enqueue_step_kernels(p, in, out);
    p->one_depth = was;
    return st;
}

ctqw_status collect_timing(ctqw_plan* p);

// Advance `count` steps.  With use_graph the sequence of (step, finalize)
// launches is captured once per (steps, starting buffer) on a private
// capture stream and the executable graph is replayed on the bound stream.
ctqw_status enqueue_steps(ctqw_plan* p, int64_t count) {
    if (count <= 0) return CTQW_OK;
    if (!p->launch.use_graph || count < 2) {
        for (int64_t s = 0; s < count; ++s) {
            ctqw_status st = enqueue_step(p);
            if (st != CTQW_OK) return st;
        }
        return CTQW_OK;
    }
    constexpr int64_t kMaxCaptured = 256;
    if (!p->cap_stream) HIP_TRY(p, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    while (count > 0) {
        const int64_t n = std::min(count, kMaxCaptured);
        const auto key = std::make_pair(n, p->cur);
        auto found = p->graphs.find(key);
        if (found == p->graphs.end()) {
            const int cur0 = p->cur;
            const int64_t done0 = p->steps_done;
            hipStream_t user = p->stream;
            const bool timing = p->timing;
            p->timing = false;               // no events inside the graph
            p->stream = p->cap_stream;
            hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
            ctqw_status st = CTQW_OK;
            if (e == hipSuccess)
                for (int64_t s = 0; s < n && st == CTQW_OK; ++s) st = enqueue_step(p);
            hipGraph_t g = nullptr;
            const hipError_t e2 = (e == hipSuccess) ? hipStreamEndCapture(p->stream, &g) : e;
            p->stream = user;
            p->timing = timing;
            p->cur = cur0;
            p->steps_done = done0;
            if (st != CTQW_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e2 != hipSuccess)
                return fail(p, CTQW_ERR_DEVICE, "step-loop capture failed: %s", hipGetErrorString(e2));
            hipGraphExec_t ex = nullptr;
            const hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e3 != hipSuccess)
                return fail(p, CTQW_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e3));
            found = p->graphs.emplace(key, ex).first;
        }
        ctqw_status st;
        if (p->timing && (st = record_event(p, 0)) != CTQW_OK) return st;
        HIP_TRY(p, hipGraphLaunch(found->second, p->stream));
        if (p->timing && (st = record_event(p, 1, n)) != CTQW_OK) return st;
        p->cur ^= (int)(n & 1);
        p->steps_done += n;
        p->have_step_stats = true;
        count -= n;
    }
    return CTQW_OK;
}

ctqw_status enqueue_observe(ctqw_plan* p, int want_pair) {
    const Layout& L = p->lay;
    if (p->prob.m == 3) {
        Obs3Args o{};
        o.psi = p->psi[p->cur];
        o.reals = at<RealDev>(p, L.reals);
        o.scale = at<double>(p, L.scale);
        o.M = at<double>(p, L.M3);
        o.occ_terms = at<double>(p, L.occ3);
        o.group_members = at<int32_t>(p, L.gmembers);
        o.group_first = at<int32_t>(p, L.gfirst);
        o.group_N = at<int32_t>(p, L.gN);
        o.group_out = at<int64_t>(p, L.gout);
        o.out = at<double>(p, L.obs);
        o.R = p->prob.R;
        o.G = (int32_t)p->group_N.size();
        o.max_N = p->max_N;
        o.want_pair = want_pair;
        HIP_TRY(p, launch_obs3(o, p->prob.dtype == CTQW_C128 ? 1 : 0, p->stream));
        return CTQW_OK;
    }
    ObsArgs o{};
    o.psi = p->psi[p->cur];
    o.reals = at<RealDev>(p, L.reals);
    o.scale = at<double>(p, L.scale);
    o.colsum = at<double>(p, L.colsum);
    o.rowsum = at<double>(p, L.rowsum);
    o.diag = at<double>(p, L.diag);
    o.site_off = at<int64_t>(p, L.site_off);
    o.group_members = at<int32_t>(p, L.gmembers);
    o.group_first = at<int32_t>(p, L.gfirst);
    o.group_N = at<int32_t>(p, L.gN);
    o.group_out = at<int64_t>(p, L.gout);
    o.out = at<double>(p, L.obs);
    o.R = p->prob.R;
    o.G = (int32_t)p->group_N.size();
    o.m = p->prob.m;
    o.max_N = p->max_N;
    o.want_pair = want_pair;
    o.dtype = p->prob.dtype == CTQW_C128 ? 1 : 0;
    HIP_TRY(p, launch_observables(o, p->stream));
    return CTQW_OK;
}

int64_t snapshot_len(const ctqw_plan* p, uint32_t obs) {
    int64_t n = 0;
    for (int32_t Ng : p->group_N) {
        if (obs & CTQW_OBS_OCCUPATION) n += Ng;
        if (obs & CTQW_OBS_PAIR) n += (int64_t)Ng * Ng;
    }
    return n;
}

// Copy the device snapshot (layout: per group [occ][pair if enabled]) into
// the caller's layout for the requested observables.
ctqw_status read_snapshot(ctqw_plan* p, uint32_t obs, double* out) {
    std::vector<double> host(p->obs_per_snapshot);
    HIP_TRY(p, hipMemcpyAsync(host.data(), p->ws + p->lay.obs.off, p->lay.obs.bytes, hipMemcpyDeviceToHost,
                              p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    int64_t k = 0;
    for (size_t g = 0; g < p->group_N.size(); ++g) {
        const int64_t Ng = p->group_N[g];
        const double* src = host.data() + p->group_out[g];
        if (obs & CTQW_OBS_OCCUPATION) {
            std::memcpy(out + k, src, Ng * 8);
            k += Ng;
        }
        if (obs & CTQW_OBS_PAIR) {
            std::memcpy(out + k, src + Ng, Ng * Ng * 8);
            k += Ng * Ng;
        }
    }
    return CTQW_OK;
}

// Sum the recorded event pairs (synchronises the stream).
ctqw_status collect_timing(ctqw_plan* p) {
    if (p->ev_used == 0) return CTQW_OK;
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    for (size_t k = 0; k + 1 < p->ev_used; k += 2) {
        float ms = 0.f;
        HIP_TRY(p, hipEventElapsedTime(&ms, p->ev[k], p->ev[k + 1]));
        p->timed_ms += ms;
        p->timed_launches += p->ev_steps[k / 2];
    }
    p->ev_used = 0;
    return CTQW_OK;
}

ctqw_status read_status(ctqw_plan* p, int32_t* st) {
    HIP_TRY(p, hipMemcpyAsync(st, p->ws + p->lay.status.off, 16, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return CTQW_OK;
}

}  // namespace

extern "C" {

const char* ctqw_version(void) { return "ctqw-mi355x 0.4 (gfx950)"; }

const char* ctqw_status_string(ctqw_status s) {
    switch (s) {
        case CTQW_OK: return "ok";
        case CTQW_ERR_INVALID_ARG: return "invalid argument";
        case CTQW_ERR_UNSUPPORTED: return "unsupported";
        case CTQW_ERR_OUT_OF_MEMORY: return "out of memory";
        case CTQW_ERR_DEVICE: return "device error";
        case CTQW_ERR_NOT_CONVERGED: return "not converged";
        case CTQW_ERR_NUMERICAL: return "numerical alarm";
        case CTQW_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

const char* ctqw_last_error(const ctqw_plan* p) {
    if (p) return p->err.c_str();
    return g_last_error.c_str();
}

ctqw_status ctqw_plan_create(const ctqw_problem* pr, ctqw_plan** out) {
    if (!pr || !out) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL problem or output pointer");
    *out = nullptr;
    if (pr->m < 1 || pr->m > 3) return fail(nullptr, CTQW_ERR_INVALID_ARG, "m must be 1, 2 or 3 (got %d)", pr->m);
    if (pr->statistics != CTQW_DISTINGUISHABLE && pr->statistics != CTQW_BOSON && pr->statistics != CTQW_FERMION)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "unknown statistics %d", pr->statistics);
    if (pr->interaction != CTQW_INT_ONSITE && pr->interaction != CTQW_INT_NEAREST)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "unknown interaction %d", pr->interaction);
    if (pr->boundary != CTQW_OPEN && pr->boundary != CTQW_PERIODIC)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "unknown boundary %d", pr->boundary);
    if (pr->dtype != CTQW_C64 && pr->dtype != CTQW_C128)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "unknown dtype %d", pr->dtype);
    if (pr->accumulation != CTQW_ACC_KAHAN && pr->accumulation != CTQW_ACC_PLAIN)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "unknown accumulation %d", pr->accumulation);
    if (pr->R < 1) return fail(nullptr, CTQW_ERR_INVALID_ARG, "R must be >= 1");
    if (!(is_fin(pr->dt) && pr->dt > 0)) return fail(nullptr, CTQW_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (pr->taylor_order < 0) return fail(nullptr, CTQW_ERR_INVALID_ARG, "taylor_order must be >= 0");
    if (!is_fin(pr->taylor_tol) || pr->taylor_tol < 0)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "taylor_tol must be finite and >= 0");
    if (pr->taylor_order == 0 && !(pr->taylor_tol > 0))
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "set taylor_order > 0 or taylor_tol > 0");
    if (pr->taylor_max_order < 0) return fail(nullptr, CTQW_ERR_INVALID_ARG, "taylor_max_order must be >= 0");
    if (!is_fin(pr->norm_alarm) || pr->norm_alarm < 0)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "norm_alarm must be finite and >= 0");
    if (pr->renormalize != 0 && pr->renormalize != 1)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "renormalize must be 0 or 1");
    if (pr->observables & ~(CTQW_OBS_OCCUPATION | CTQW_OBS_PAIR))
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "unknown observable bits 0x%x", pr->observables);
    if (pr->n_sites == 0 && !pr->n_sites_per_real)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "set n_sites or n_sites_per_real");
    if (pr->n_sites < 0) return fail(nullptr, CTQW_ERR_INVALID_ARG, "n_sites must be >= 0");
    if (pr->R > 65535) return fail(nullptr, CTQW_ERR_UNSUPPORTED, "at most 65535 realisations per plan");
    if (pr->m == 3 && pr->statistics != CTQW_DISTINGUISHABLE)
        return fail(nullptr, CTQW_ERR_UNSUPPORTED, "three bosons are not built");
    if (pr->m == 3 && (pr->n_sites <= 0 || pr->n_sites > 1024))
        return fail(nullptr, CTQW_ERR_UNSUPPORTED, "three particles need one lattice size N <= 1024");
    if (pr->statistics == CTQW_BOSON && pr->m != 2 && pr->m != 1)
        return fail(nullptr, CTQW_ERR_UNSUPPORTED, "bosons are built for m == 2");
    if (pr->statistics == CTQW_BOSON && pr->m == 2 && pr->boundary == CTQW_PERIODIC)
        return fail(nullptr, CTQW_ERR_UNSUPPORTED, "bosons on a ring are not built (use distinguishable "
                                                   "particles with a symmetrised start)");
    if (pr->statistics == CTQW_FERMION && pr->m != 2 && pr->m != 1)
        return fail(nullptr, CTQW_ERR_UNSUPPORTED, "fermions are built for m == 2");
    if (pr->statistics == CTQW_FERMION && pr->m == 2 && pr->boundary == CTQW_PERIODIC)
        return fail(nullptr, CTQW_ERR_UNSUPPORTED, "fermions on a ring are not built on the chain path (the wrap "
                                                   "bond crosses the stored triangle; use the pair graph)");

    ctqw_plan* p = new (std::nothrow) ctqw_plan();
    if (!p) return fail(nullptr, CTQW_ERR_OUT_OF_MEMORY, "host allocation failed");
    try {
        p->prob = *pr;
        p->prob.n_sites_per_real = nullptr;
        const int64_t R = pr->R;
        p->N.resize(R);
        for (int64_t r = 0; r < R; ++r) {
            const int N = pr->n_sites > 0 ? pr->n_sites : pr->n_sites_per_real[r];
            if (N < 2 || N > kMaxSites) {
                delete p;
                return fail(nullptr, CTQW_ERR_INVALID_ARG, "realisation %lld: N = %d outside [2, %d]",
                            (long long)r, N, kMaxSites);
            }
            if (pr->boundary == CTQW_PERIODIC && N < 3) {
                delete p;
                return fail(nullptr, CTQW_ERR_INVALID_ARG, "a ring needs N >= 3");
            }
            p->N[r] = N;
        }
        p->state_off.resize(R + 1);
        p->param_off.resize(R);
        p->site_off.resize(R);
        int64_t so = 0, po = 0, st = 0;
        for (int64_t r = 0; r < R; ++r) {
            p->state_off[r] = so;
            const int64_t a = amplitudes(*pr, p->N[r]);
            if (so > INT64_MAX / 16 - a) {
                delete p;
                return fail(nullptr, CTQW_ERR_OUT_OF_MEMORY, "state size overflows");
            }
            so += a;
            p->param_off[r] = (int32_t)po;
            po += p->N[r];
            p->site_off[r] = st;
            st += p->N[r];
            p->max_N = std::max(p->max_N, p->N[r]);
        }
        p->state_off[R] = so;
        p->zero_block = (int32_t)po;
        po += p->max_N;
        if (po > INT32_MAX) {
            delete p;
            return fail(nullptr, CTQW_ERR_OUT_OF_MEMORY, "parameter tables too large");
        }
        p->param_total = po;
        p->site_total = st;
        p->Jpad.assign(po, 0.0);
        p->Epad.assign(po, 0.0);
        // groups of equal N, ascending
        std::map<int32_t, std::vector<int32_t>> groups;
        for (int64_t r = 0; r < R; ++r) groups[p->N[r]].push_back((int32_t)r);
        int64_t go = 0;
        p->group_first.push_back(0);
        for (auto& kv : groups) {
            p->group_N.push_back(kv.first);
            for (int32_t r : kv.second) p->group_members.push_back(r);
            p->group_first.push_back((int32_t)p->group_members.size());
            p->group_out.push_back(go);
            go += kv.first;
            if (pr->observables & CTQW_OBS_PAIR) go += (int64_t)kv.first * kv.first;
        }
        p->obs_per_snapshot = go;
        p->launch.cols_per_lane = 1;
        p->launch.waves_per_block = 4;
        p->launch.persistent = 0;
        p->launch.use_graph = 0;
        p->launch.waves_per_cu = 0;
        p->launch.chunked = 0;
        p->launch.band_align = 128;
        p->launch.terms_per_pass = 0;
        p->launch.band_mode = 0;
        p->launch.row_segments = 0;
        p->launch.three_form = 0;
        p->order.assign(R, 0);
        p->xbound.assign(R, 0.0);
    } catch (const std::bad_alloc&) {
        delete p;
        return fail(nullptr, CTQW_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    *out = p;
    return CTQW_OK;
}

ctqw_status ctqw_plan_destroy(ctqw_plan* p) {
    delete p;
    return CTQW_OK;
}

ctqw_status ctqw_set_params(ctqw_plan* p, const double* J, const double* eps, const double* U) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!J || !eps || !U) return fail(p, CTQW_ERR_INVALID_ARG, "NULL parameter array");
    const ctqw_problem& pr = p->prob;
    const int64_t R = pr.R;
    int64_t nJ = 0, nE = 0;
    for (int64_t r = 0; r < R; ++r) {
        nJ += n_bonds(pr, p->N[r]);
        nE += p->N[r];
    }
    for (int64_t k = 0; k < nJ; ++k)
        if (!is_fin(J[k])) return fail(p, CTQW_ERR_INVALID_ARG, "J[%lld] is not finite", (long long)k);
    for (int64_t k = 0; k < nE; ++k)
        if (!is_fin(eps[k])) return fail(p, CTQW_ERR_INVALID_ARG, "eps[%lld] is not finite", (long long)k);
    for (int64_t r = 0; r < R; ++r)
        if (!is_fin(U[r])) return fail(p, CTQW_ERR_INVALID_ARG, "U[%lld] is not finite", (long long)r);

    std::vector<int32_t> order(R);
    std::vector<double> xb(R);
    std::vector<double> Jpad(p->param_total, 0.0), Epad(p->param_total, 0.0);
    const int cap = max_order_cap(pr);
    int64_t jo = 0, eo = 0;
    for (int64_t r = 0; r < R; ++r) {
        const int N = p->N[r];
        const int nb = n_bonds(pr, N);
        const int32_t po = p->param_off[r];
        for (int i = 0; i < nb; ++i) Jpad[po + i] = J[jo + i];
        for (int i = 0; i < N; ++i) Epad[po + i] = eps[eo + i];
        jo += nb;
        eo += N;
        // switching noise: every bond's |J| may reach |Jbar| + a
        double gmax = 0.0;
        auto absJ = [&](int b) { return b < nb ? std::fabs(Jpad[po + b]) + p->tele_amp : 0.0; };
        for (int i = 0; i < N; ++i) {
            const double jl = absJ((i + N - 1) % N);
            const double jr = absJ(i);
            gmax = std::max(gmax, std::fabs(Epad[po + i]) + jl + jr);
        }
        const double G = pr.m * gmax + (pr.m > 1 ? std::fabs(U[r]) * pr.m * (pr.m - 1) / 2.0 : 0.0);
        const double x = G * pr.dt;
        int n;
        if (pr.taylor_order > 0) {
            n = pr.taylor_order;
            if (n > cap)
                return fail(p, CTQW_ERR_NOT_CONVERGED, "taylor_order %d above the cap %d", n, cap);
        } else {
            n = 1;
            while (remainder_bound(x, n) > pr.taylor_tol) {
                ++n;
                if (n > cap)
                    return fail(p, CTQW_ERR_NOT_CONVERGED,
                                "realisation %lld: dt*||H|| <= %.4g needs more than %d Taylor terms for tol %.3g",
                                (long long)r, x, cap, pr.taylor_tol);
            }
        }
        order[r] = n;
        xb[r] = x;
    }
    p->J.assign(J, J + nJ);
    p->eps.assign(eps, eps + nE);
    p->U.assign(U, U + R);
    p->Jpad.swap(Jpad);
    p->Epad.swap(Epad);
    p->order.swap(order);
    p->xbound.swap(xb);
    p->params_set = true;
    return build_tables(p);
}

ctqw_status ctqw_draw_params(ctqw_plan* p, const double* J_base, const double* eps_base, double U_base,
                             const ctqw_noise* J_noise, const ctqw_noise* eps_noise, const ctqw_noise* U_noise,
                             uint64_t seed) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    const ctqw_problem& pr = p->prob;
    const ctqw_noise none{CTQW_DIST_NONE, 0.0, 0.0};
    const ctqw_noise* noises[3] = {J_noise ? J_noise : &none, eps_noise ? eps_noise : &none,
                                   U_noise ? U_noise : &none};
    for (const ctqw_noise* n : noises) {
        if (n->dist != CTQW_DIST_NONE && n->dist != CTQW_DIST_UNIFORM && n->dist != CTQW_DIST_NORMAL)
            return fail(p, CTQW_ERR_INVALID_ARG, "unknown noise distribution %d", n->dist);
        if (!is_fin(n->a) || !is_fin(n->b)) return fail(p, CTQW_ERR_INVALID_ARG, "non-finite noise parameter");
    }
    if (!is_fin(U_base)) return fail(p, CTQW_ERR_INVALID_ARG, "non-finite U_base");
    const int nb_max = n_bonds(pr, p->max_N);
    if (J_base)
        for (int i = 0; i < nb_max; ++i)
            if (!is_fin(J_base[i])) return fail(p, CTQW_ERR_INVALID_ARG, "J_base[%d] is not finite", i);
    if (eps_base)
        for (int i = 0; i < p->max_N; ++i)
            if (!is_fin(eps_base[i])) return fail(p, CTQW_ERR_INVALID_ARG, "eps_base[%d] is not finite", i);
    std::vector<double> J, eps, U(pr.R);
    for (int64_t r = 0; r < pr.R; ++r) {
        const int N = p->N[r];
        const int nb = n_bonds(pr, N);
        for (int i = 0; i < nb; ++i)
            J.push_back((J_base ? J_base[i] : 1.0) + noise_draw(*noises[0], seed, r, NOISE_BOND, i));
        for (int i = 0; i < N; ++i)
            eps.push_back((eps_base ? eps_base[i] : 0.0) + noise_draw(*noises[1], seed, r, NOISE_SITE, i));
        U[r] = U_base + noise_draw(*noises[2], seed, r, NOISE_INTERACTION, 0);
    }
    return ctqw_set_params(p, J.data(), eps.data(), U.data());
}

ctqw_status ctqw_get_params(const ctqw_plan* p, double* J, double* eps, double* U) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!p->params_set) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_STATE, "parameters not set");
    if (J) std::memcpy(J, p->J.data(), p->J.size() * 8);
    if (eps) std::memcpy(eps, p->eps.data(), p->eps.size() * 8);
    if (U) std::memcpy(U, p->U.data(), p->U.size() * 8);
    return CTQW_OK;
}

ctqw_status ctqw_orders(const ctqw_plan* p, int32_t* orders) {
    if (!p || !orders) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_INVALID_ARG, "NULL argument");
    if (!p->params_set) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_STATE, "parameters not set");
    std::memcpy(orders, p->order.data(), p->order.size() * 4);
    return CTQW_OK;
}

ctqw_status ctqw_layout(const ctqw_plan* p, int64_t* offsets) {
    if (!p || !offsets) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_INVALID_ARG, "NULL argument");
    std::memcpy(offsets, p->state_off.data(), p->state_off.size() * 8);
    return CTQW_OK;
}

ctqw_status ctqw_groups(const ctqw_plan* p, int32_t* n_groups, int32_t* sizes) {
    if (!p || !n_groups) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_INVALID_ARG, "NULL argument");
    *n_groups = (int32_t)p->group_N.size();
    if (sizes) std::memcpy(sizes, p->group_N.data(), p->group_N.size() * 4);
    return CTQW_OK;
}

}  // extern "C"

namespace {
// Stored amplitudes of the realisations of group g (all equal).
int64_t group_dim(const ctqw_plan* p, int32_t g) {
    const int32_t r = p->group_members[p->group_first[g]];
    return p->state_off[r + 1] - p->state_off[r];
}
}  // namespace

extern "C" {

ctqw_status ctqw_set_telegraph(ctqw_plan* p, double amplitude, double rate, uint64_t seed) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!is_fin(amplitude) || amplitude < 0.0 || !is_fin(rate) || rate < 0.0)
        return fail(p, CTQW_ERR_INVALID_ARG, "amplitude and rate must be finite and >= 0");
    const double a0 = p->tele_amp, r0 = p->tele_rate;
    const uint64_t s0 = p->tele_seed;
    p->tele_amp = amplitude;
    p->tele_rate = rate;
    p->tele_seed = seed;
    if (p->params_set) {
        // orders follow the largest |J|; the tables (and the signs) are
        // uploaded again, so the switching process starts anew
        const std::vector<double> J = p->J, eps = p->eps, U = p->U;
        const ctqw_status st = ctqw_set_params(p, J.data(), eps.data(), U.data());
        if (st != CTQW_OK) {
            p->tele_amp = a0;
            p->tele_rate = r0;
            p->tele_seed = s0;
            (void)ctqw_set_params(p, J.data(), eps.data(), U.data());
            return st;
        }
    }
    return CTQW_OK;
}

ctqw_status ctqw_density_workspace(const ctqw_plan* p, int32_t group, int64_t* bytes) {
    if (!p || !bytes) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_INVALID_ARG, "NULL argument");
    if (!p->params_set) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_STATE, "parameters not set");
    if (group < 0 || group >= (int32_t)p->group_N.size())
        return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_INVALID_ARG, "group %d out of range", group);
    const int64_t Rg = p->group_first[group + 1] - p->group_first[group];
    const int dtype = p->prob.dtype == CTQW_C128 ? 1 : 0;
    const int64_t tile = herk_tile(dtype), stage = herk_stage(dtype);
    const int64_t Dp = (group_dim(p, group) + tile - 1) / tile * tile, Rp = (Rg + stage - 1) / stage * stage;
    *bytes = 2 * Dp * Rp * (dtype ? 8 : 4);   // real and imaginary planes, zero padded
    return CTQW_OK;
}

ctqw_status ctqw_density_matrix(ctqw_plan* p, int32_t group, void* rho, int64_t ld, int32_t lower_only,
                                void* workspace, int64_t workspace_bytes) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!rho || !workspace) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    int64_t need = 0;
    ctqw_status st = ctqw_density_workspace(p, group, &need);
    if (st != CTQW_OK) return st;
    const int64_t D = group_dim(p, group);
    const int64_t Rg = p->group_first[group + 1] - p->group_first[group];
    if (ld < D) return fail(p, CTQW_ERR_INVALID_ARG, "ld %lld below the dimension %lld", (long long)ld, (long long)D);
    if (workspace_bytes < need)
        return fail(p, CTQW_ERR_INVALID_ARG, "workspace too small (%lld < %lld bytes)", (long long)workspace_bytes,
                    (long long)need);
    if (D > INT32_MAX || ld > INT32_MAX || Rg > 65535)
        return fail(p, CTQW_ERR_UNSUPPORTED, "density matrix limited to D, ld < 2^31 and 65535 realisations");
    if ((st = ensure_ready(p)) != CTQW_OK) return st;
    const int dtype = p->prob.dtype == CTQW_C128 ? 1 : 0;
    DensityArgs a{};
    a.psi = p->psi[p->cur];
    a.reals = at<RealDev>(p, p->lay.reals);
    a.scale = at<double>(p, p->lay.scale);
    a.members = at<int32_t>(p, p->lay.gmembers) + p->group_first[group];
    a.A = workspace;
    a.D = D;
    a.R_g = Rg;
    a.triangle = (p->prob.m == 2 && p->prob.statistics != CTQW_DISTINGUISHABLE) ? 1 : 0;
    const int64_t tile = herk_tile(dtype), stage = herk_stage(dtype);
    a.Dp = (D + tile - 1) / tile * tile;
    a.Rp = (Rg + stage - 1) / stage * stage;
    HIP_TRY(p, launch_density_gather(a, dtype, p->stream));
    HerkArgs h{};
    h.G = workspace;
    h.rho = rho;
    h.D = D;
    h.Dp = a.Dp;
    h.ld = ld;
    h.Rp = (int32_t)a.Rp;
    const int64_t T = a.Dp / tile;
    h.n_tiles = T * (T + 1) / 2;
    h.inv_R = 1.0 / (double)Rg;
    HIP_TRY(p, launch_herk(h, dtype, p->stream));
    if (!lower_only) HIP_TRY(p, launch_density_mirror(rho, D, ld, dtype, p->stream));
    return CTQW_OK;
}

ctqw_status ctqw_graph_tables(int32_t n_nodes, int32_t n_edges, const int32_t* edges, int32_t m, int32_t statistics,
                              int32_t R, const double* J, const double* eps, const double* U, int32_t* n_states,
                              int32_t* width, int32_t* nbr, double* hop, double* onsite) {
    if (n_nodes < 1 || n_edges < 0 || R < 0)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "n_nodes must be positive, n_edges and R >= 0");
    if (m != 1 && m != 2) return fail(nullptr, CTQW_ERR_INVALID_ARG, "m must be 1 or 2 (got %d)", m);
    if (statistics != CTQW_DISTINGUISHABLE && statistics != CTQW_BOSON && statistics != CTQW_FERMION)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "unknown statistics %d", statistics);
    if (!n_states || !width || (n_edges > 0 && !edges))
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL argument");
    const int64_t n = n_nodes;
    // One-particle slots: each bond fills one slot of both of its nodes, in
    // bond order, the first endpoint's slot first.
    std::vector<int32_t> deg(n, 0);
    std::vector<std::pair<int64_t, int64_t>> seen;
    seen.reserve(n_edges);
    for (int64_t e = 0; e < n_edges; ++e) {
        const int64_t a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || a >= n || b < 0 || b >= n) return fail(nullptr, CTQW_ERR_INVALID_ARG, "bond %lld: node out of range", (long long)e);
        if (a == b) return fail(nullptr, CTQW_ERR_INVALID_ARG, "bond %lld is a self-loop (use the on-site energies)", (long long)e);
        seen.emplace_back(std::min(a, b), std::max(a, b));
        ++deg[a];
        ++deg[b];
    }
    {
        std::vector<std::pair<int64_t, int64_t>> sorted_b(seen);
        std::sort(sorted_b.begin(), sorted_b.end());
        if (std::adjacent_find(sorted_b.begin(), sorted_b.end()) != sorted_b.end())
            return fail(nullptr, CTQW_ERR_INVALID_ARG, "repeated bond");
    }
    const int32_t w1 = n_edges ? *std::max_element(deg.begin(), deg.end()) : 0;
    std::vector<int32_t> nbr1((size_t)w1 * n, -1), bond1((size_t)w1 * n, -1), fill(n, 0);
    for (int64_t e = 0; e < n_edges; ++e) {
        const int32_t a = edges[2 * e], b = edges[2 * e + 1];
        int32_t k = fill[a]++;
        nbr1[(size_t)k * n + a] = b;
        bond1[(size_t)k * n + a] = (int32_t)e;
        k = fill[b]++;
        nbr1[(size_t)k * n + b] = a;
        bond1[(size_t)k * n + b] = (int32_t)e;
    }
    // States: one node (m = 1); ordered pairs a * n + b (distinguishable);
    // pairs a <= b (bosons) or a < b (fermions) in lexicographic order.
    const bool boson = m == 2 && statistics == CTQW_BOSON, fermion = m == 2 && statistics == CTQW_FERMION;
    int64_t D = m == 1 ? n : (boson ? n * (n + 1) / 2 : (fermion ? n * (n - 1) / 2 : n * n));
    const int64_t W = m == 1 ? w1 : 2 * (int64_t)w1;
    if (D < 1 || D > INT32_MAX || W * D > INT32_MAX)
        return fail(nullptr, CTQW_ERR_UNSUPPORTED, "%lld states x %lld slots exceed the 32-bit tables", (long long)D, (long long)W);
    *n_states = (int32_t)D;
    *width = (int32_t)W;
    if (!nbr && !hop && !onsite) return CTQW_OK;   // sizes only
    if (!nbr || !hop || !onsite || (R > 0 && ((n_edges > 0 && !J) || !eps || (m == 2 && !U))))
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL table or parameter array");
    for (int64_t k = 0; k < (int64_t)R * n_edges; ++k)
        if (!std::isfinite(J[k])) return fail(nullptr, CTQW_ERR_INVALID_ARG, "non-finite hopping");
    for (int64_t k = 0; k < (int64_t)R * n; ++k)
        if (!std::isfinite(eps[k])) return fail(nullptr, CTQW_ERR_INVALID_ARG, "non-finite on-site energy");
    if (m == 2)
        for (int64_t r = 0; r < R; ++r)
            if (!std::isfinite(U[r])) return fail(nullptr, CTQW_ERR_INVALID_ARG, "non-finite U");
    auto index = [&](int64_t a, int64_t b) -> int64_t {
        if (!boson && !fermion) return a * n + b;
        const int64_t lo = std::min(a, b), hi = std::max(a, b);
        return boson ? lo * n - lo * (lo - 1) / 2 + (hi - lo) : lo * n - lo * (lo + 1) / 2 + (hi - lo - 1);
    };
    // state k -> its nodes (A, B)
    std::vector<int32_t> SA(D), SB(D);
    {
        int64_t k = 0;
        if (m == 1) {
            for (int64_t a = 0; a < n; ++a) { SA[k] = (int32_t)a; SB[k] = (int32_t)a; ++k; }
        } else {
            for (int64_t a = 0; a < n; ++a)
                for (int64_t b = boson ? a : (fermion ? a + 1 : 0); b < n; ++b) { SA[k] = (int32_t)a; SB[k] = (int32_t)b; ++k; }
        }
    }
    // slot (half, k) of state s: the particle `mover` (A for half 0, B for 1)
    // steps along its node's slot k; factor f multiplies the bond's J
    std::vector<int32_t> sbond((size_t)W * D, -1);
    std::vector<double> sfac((size_t)W * D, 0.0);
    for (int64_t st = 0; st < D; ++st) {
        const int64_t A = SA[st], B = SB[st];
        for (int half = 0; half < (m == 1 ? 1 : 2); ++half) {
            const int64_t mover = half == 0 ? A : B, still = half == 0 ? B : A;
            for (int32_t k = 0; k < w1; ++k) {
                const size_t slot = (size_t)(half * w1 + k) * D + st;
                const int64_t c = nbr1[(size_t)k * n + mover];
                if (c < 0) continue;
                if (fermion && c == still) continue;          // no two fermions on one node
                int64_t tgt;
                double f = 1.0;
                if (m == 1) {
                    tgt = c;
                } else {
                    tgt = half == 0 ? index(c, still) : index(still, c);
                    if (boson) f = (A == B) ? 1.0 / std::sqrt(2.0) : (c == still ? std::sqrt(2.0) : 1.0);
                    // a fermion move that carries the mover past the other particle flips the pair's order
                    if (fermion) f = ((c < still) == (mover < still)) ? 1.0 : -1.0;
                }
                nbr[slot] = (int32_t)tgt;
                sbond[slot] = bond1[(size_t)k * n + mover];
                sfac[slot] = f;
            }
        }
    }
    for (size_t slot = 0; slot < (size_t)W * D; ++slot)
        if (sbond[slot] < 0) nbr[slot] = -1;
    for (int64_t r = 0; r < R; ++r) {
        double* h = hop + (size_t)r * W * D;
        for (size_t slot = 0; slot < (size_t)W * D; ++slot)
            h[slot] = sbond[slot] >= 0 ? J[(size_t)r * n_edges + sbond[slot]] * sfac[slot] : 0.0;
        double* o = onsite + (size_t)r * D;
        const double* er = eps + (size_t)r * n;
        for (int64_t st = 0; st < D; ++st) {
            if (m == 1) o[st] = er[SA[st]];
            else o[st] = er[SA[st]] + er[SB[st]] + (SA[st] == SB[st] ? U[r] : 0.0);
        }
    }
    return CTQW_OK;
}

ctqw_status ctqw_graph_workspace(int32_t n_nodes, int32_t R, int32_t dtype, int64_t* bytes) {
    if (!bytes) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL argument");
    if (n_nodes < 1 || R < 1)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "n_nodes and R must be positive (got %d, %d)", n_nodes, R);
    if (dtype != CTQW_C64 && dtype != CTQW_C128) return fail(nullptr, CTQW_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    // two term buffers and the partial sum
    *bytes = 3 * (int64_t)n_nodes * (int64_t)R * (dtype == CTQW_C128 ? 16 : 8);
    return CTQW_OK;
}

ctqw_status ctqw_graph_orders(int32_t n_nodes, int32_t width, const int32_t* nbr, const double* hop,
                              const double* onsite, int32_t R, double dt, double tol, int32_t max_order,
                              int32_t* orders) {
    if (n_nodes < 1 || R < 1 || width < 0)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "n_nodes, R must be positive and width >= 0");
    if (!onsite || !orders || (width > 0 && (!nbr || !hop))) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL argument");
    if (!std::isfinite(dt) || !(tol > 0.0) || !std::isfinite(tol))
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "dt must be finite and tol positive");
    if (max_order < 1 || max_order > 64) return fail(nullptr, CTQW_ERR_INVALID_ARG, "max_order must be in 1..64");
    const int64_t n = n_nodes;
    for (int64_t r = 0; r < R; ++r) {
        // Gershgorin: ||H_r||_2 <= max_i (|H_ii| + sum_k |H_i,nbr(k,i)|)
        double G = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double row = std::fabs(onsite[r * n + i]);
            for (int64_t k = 0; k < width; ++k) {
                const int32_t j = nbr[k * n + i];
                if (j >= 0 && j < n_nodes) row += std::fabs(hop[(r * width + k) * n + i]);
            }
            if (!std::isfinite(row)) return fail(nullptr, CTQW_ERR_INVALID_ARG, "non-finite table entry");
            G = std::max(G, row);
        }
        const double x = std::fabs(dt) * G;
        // smallest n with x^(n+1)/(n+1)! / (1 - x/(n+2)) <= tol
        double term = x;   // x^(n+1)/(n+1)! for n = 0
        int32_t ord = 0;
        for (int32_t k = 1; k <= max_order; ++k) {
            term *= x / (double)(k + 1);
            if (x < k + 2 && term / (1.0 - x / (k + 2)) <= tol) {
                ord = k;
                break;
            }
        }
        if (ord == 0)
            return fail(nullptr, CTQW_ERR_NOT_CONVERGED, "realisation %lld needs more than %d terms (x = %g)",
                        (long long)r, max_order, x);
        orders[r] = ord;
    }
    return CTQW_OK;
}

ctqw_status ctqw_graph_evolve(int32_t n_nodes, int32_t width, const int32_t* nbr, const void* hop, const void* onsite,
                              int32_t R, int32_t dtype, double dt, int32_t order, int64_t n_steps, void* psi,
                              void* workspace, int64_t workspace_bytes, double* norms, void* hip_stream) {
    int64_t need = 0;
    ctqw_status st = ctqw_graph_workspace(n_nodes, R, dtype, &need);
    if (st != CTQW_OK) return st;
    if (width < 0) return fail(nullptr, CTQW_ERR_INVALID_ARG, "width must be >= 0 (got %d)", width);
    if (!onsite || !psi || !workspace || (width > 0 && (!nbr || !hop)))
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL argument");
    if (!std::isfinite(dt)) return fail(nullptr, CTQW_ERR_INVALID_ARG, "dt must be finite");
    constexpr int32_t kGraphMaxOrder = 64;   // one pass per term, no pipeline depth limit
    if (order < 1 || order > kGraphMaxOrder)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "order must be in 1..%d (got %d)", kGraphMaxOrder, order);
    if (n_steps < 0) return fail(nullptr, CTQW_ERR_INVALID_ARG, "n_steps must be >= 0");
    if (workspace_bytes < need)
        return fail(nullptr, CTQW_ERR_INVALID_ARG, "workspace too small (%lld < %lld bytes)",
                    (long long)workspace_bytes, (long long)need);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int dt_ = dtype == CTQW_C128 ? 1 : 0;
    const int64_t esz = dt_ ? 16 : 8;
    const int64_t bytes = (int64_t)n_nodes * R * esz;
    char* ws = static_cast<char*>(workspace);
    void* T[2] = {ws, ws + bytes};
    void* acc = ws + 2 * bytes;
    for (int64_t step = 0; step < n_steps; ++step) {
        GraphTermArgs a{};
        a.nbr = nbr;
        a.hop = hop;
        a.onsite = onsite;
        a.n = n_nodes;
        a.width = width;
        a.R = R;
        a.src = psi;
        a.acc_in = psi;
        for (int32_t j = 1; j <= order; ++j) {
            const bool last = j == order;
            a.t_out = last ? nullptr : T[(j - 1) & 1];
            // the last term may write the state: it reads only the previous term and the sum
            a.acc_out = (last && order > 1) ? psi : acc;
            a.c = dt / (double)j;
            HIP_TRY(nullptr, launch_graph_term(a, dt_, s));
            a.src = a.t_out;
            a.acc_in = acc;
        }
        if (order == 1) HIP_TRY(nullptr, hipMemcpyAsync(psi, acc, bytes, hipMemcpyDeviceToDevice, s));
        if (norms) HIP_TRY(nullptr, launch_graph_norms(psi, n_nodes, R, norms + step * (int64_t)R, dt_, s));
    }
    return CTQW_OK;
}

ctqw_status ctqw_sizes(const ctqw_plan* p, int64_t* state_bytes, int64_t* workspace_bytes) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!p->params_set) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_STATE, "parameters not set");
    const int64_t esz = p->prob.dtype == CTQW_C128 ? 16 : 8;
    if (state_bytes) *state_bytes = p->state_off.back() * esz;
    if (workspace_bytes) *workspace_bytes = p->lay.total;
    return CTQW_OK;
}

ctqw_status ctqw_work_items(const ctqw_plan* p, int64_t* items, int64_t* waves) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!p->params_set) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_STATE, "parameters not set");
    const int64_t n = p->prob.m == 3 ? p->n_parts : (int64_t)p->items.size();
    if (items) *items = n;
    if (waves) {
        *waves = p->prob.m == 3 ? n * 8 : n;
        if (p->prob.m != 3 && !p->launch.persistent) {
            // regular: whole blocks of waves_per_block waves per launch (the
            // largest of the per-order launches)
            const int64_t wpb = p->launch.waves_per_block;
            auto whole = [&](int64_t k) { return (k + wpb - 1) / wpb * wpb; };
            *waves = whole(n);
            if (!p->chunk && !p->order_runs.empty()) {
                *waves = 0;
                for (const auto& run : p->order_runs) *waves = std::max<int64_t>(*waves, whole(run[2] - run[1]));
            }
        }
        if (p->prob.m != 3 && p->launch.persistent && p->bound) {
            // the persistent grid: resident waves of the device (the
            // largest of the per-order launches)
            ctqw_plan* q = const_cast<ctqw_plan*>(p);
            StepConfig c = step_config(q);
            c.vec = (!p->chunk && p->all_vec) ? 1 : 0;
            int n_waves = 0;
            ctqw_status st = grid_for(q, c, &n_waves);
            if (st != CTQW_OK) return st;
            if (!p->chunk && !p->order_runs.empty()) {
                n_waves = 0;
                for (const auto& run : p->order_runs) {
                    StepConfig cr = step_config(q);
                    cr.levels = run[0];
                    cr.vec = run[3];
                    cr.two = run[4];
                    int w = 0;
                    if ((st = grid_for(q, cr, &w, run[2] - run[1])) != CTQW_OK) return st;
                    n_waves = std::max(n_waves, w);
                }
            }
            *waves = n_waves;
        }
    }
    return CTQW_OK;
}

ctqw_status ctqw_get_launch(const ctqw_plan* p, ctqw_launch* out) {
    if (!p || !out) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_INVALID_ARG, "NULL argument");
    *out = p->launch;
    return CTQW_OK;
}

ctqw_status ctqw_set_launch(ctqw_plan* p, const ctqw_launch* l) {
    if (!p || !l) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    if (l->cols_per_lane != 1 && l->cols_per_lane != 2)
        return fail(p, CTQW_ERR_INVALID_ARG, "cols_per_lane must be 1 or 2");
    if (l->waves_per_block != 1 && l->waves_per_block != 2 && l->waves_per_block != 4)
        return fail(p, CTQW_ERR_INVALID_ARG, "waves_per_block must be 1, 2 or 4");
    if ((l->persistent != 0 && l->persistent != 1) || (l->use_graph != 0 && l->use_graph != 1) ||
        l->waves_per_cu < 0 || (l->chunked != 0 && l->chunked != 1))
        return fail(p, CTQW_ERR_INVALID_ARG, "bad persistent / use_graph / waves_per_cu / chunked");
    if (l->band_align != 0 && l->band_align != 64 && l->band_align != 128 && l->band_align != 256)
        return fail(p, CTQW_ERR_INVALID_ARG, "band_align must be 0, 64, 128 or 256 bytes");
    if (l->terms_per_pass < 0 || l->terms_per_pass > 3)
        return fail(p, CTQW_ERR_INVALID_ARG, "terms_per_pass must be 0 (default) or 1..3");
    if (l->band_mode != 0 && l->band_mode != 1)
        return fail(p, CTQW_ERR_INVALID_ARG, "band_mode must be 0 (output-aligned) or 1 (window-aligned)");
    if (l->three_form != 0 && l->three_form != 1)
        return fail(p, CTQW_ERR_INVALID_ARG, "three_form must be 0 (chained sum) or 1 (product form)");
    if (l->row_segments < 0 || l->row_segments > kMaxRowSegments)
        return fail(p, CTQW_ERR_INVALID_ARG, "row_segments must be 0 (auto), 1 (never split) or 2..%d", kMaxRowSegments);
    const ctqw_launch old = p->launch;
    p->launch = *l;
    if (p->params_set) {
        ctqw_status st = build_tables(p);
        if (st != CTQW_OK) {
            p->launch = old;
            build_tables(p);
            return st;
        }
    }
    return CTQW_OK;
}

ctqw_status ctqw_bind(ctqw_plan* p, void* psi_a, void* psi_b, int64_t state_bytes, void* workspace,
                      int64_t workspace_bytes, void* hip_stream) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!p->params_set) return fail(p, CTQW_ERR_STATE, "set parameters before binding");
    if (!psi_a || !psi_b || !workspace) return fail(p, CTQW_ERR_INVALID_ARG, "NULL device buffer");
    if (psi_a == psi_b) return fail(p, CTQW_ERR_INVALID_ARG, "the two state buffers must differ");
    const int64_t esz = p->prob.dtype == CTQW_C128 ? 16 : 8;
    if (state_bytes < p->state_off.back() * esz)
        return fail(p, CTQW_ERR_INVALID_ARG, "state buffers too small (%lld < %lld bytes)", (long long)state_bytes,
                    (long long)(p->state_off.back() * esz));
    if (workspace_bytes < p->lay.total)
        return fail(p, CTQW_ERR_INVALID_ARG, "workspace too small (%lld < %lld bytes)", (long long)workspace_bytes,
                    (long long)p->lay.total);
    if ((reinterpret_cast<uintptr_t>(psi_a) | reinterpret_cast<uintptr_t>(psi_b) |
         reinterpret_cast<uintptr_t>(workspace)) & 255)
        return fail(p, CTQW_ERR_INVALID_ARG, "device buffers must be 256-byte aligned");
    int dev = 0;
    HIP_TRY(p, hipGetDevice(&dev));
    HIP_TRY(p, hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, dev));
    p->psi[0] = psi_a;
    p->psi[1] = psi_b;
    p->cur = 0;
    p->ws = static_cast<uint8_t*>(workspace);
    p->ws_bytes = workspace_bytes;
    p->state_bytes_bound = state_bytes;
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->bound = true;
    p->drop_graphs();
    p->tables_dirty = true;
    ctqw_status st = upload_tables(p);
    if (st != CTQW_OK) {
        p->bound = false;
        return st;
    }
    return CTQW_OK;
}

ctqw_status ctqw_init_product_state(ctqw_plan* p, const int32_t* sites, int32_t per_real) {
    if (!p || !sites) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    const ctqw_problem& pr = p->prob;
    const int64_t cnt = per_real ? pr.R * pr.m : pr.m;
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t r = per_real ? k / pr.m : 0;
        if (sites[k] < 0 || sites[k] >= p->N[per_real ? r : 0])
            return fail(p, CTQW_ERR_INVALID_ARG, "start site %d out of range", sites[k]);
    }
    if (!per_real)
        for (int64_t r = 0; r < pr.R; ++r)
            for (int a = 0; a < pr.m; ++a)
                if (sites[a] >= p->N[r])
                    return fail(p, CTQW_ERR_INVALID_ARG, "start site %d out of range for N = %d", sites[a], p->N[r]);
    if (pr.statistics == CTQW_FERMION && pr.m == 2)
        for (int64_t k = 0; k < cnt; k += 2)
            if (sites[k] == sites[k + 1])
                return fail(p, CTQW_ERR_INVALID_ARG, "two fermions on node %d", sites[k]);
    HIP_TRY(p, hipMemcpyAsync(p->ws + p->lay.sites.off, sites, cnt * 4, hipMemcpyHostToDevice, p->stream));
    InitArgs a{};
    a.psi = p->psi[0];
    a.reals = at<RealDev>(p, p->lay.reals);
    a.sites = at<int32_t>(p, p->lay.sites);
    a.per_real = per_real ? 1 : 0;
    a.m = pr.m;
    a.R = pr.R;
    a.total = p->state_off.back();
    a.dtype = pr.dtype == CTQW_C128 ? 1 : 0;
    HIP_TRY(p, launch_init(a, p->stream));
    std::vector<double> ones(pr.R, 1.0);
    HIP_TRY(p, hipMemcpyAsync(p->ws + p->lay.scale.off, ones.data(), pr.R * 8, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(p, launch_fill_zero(p->ws + p->lay.status.off, 16, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->cur = 0;
    p->steps_done = 0;
    p->have_step_stats = false;
    p->grad_ws = nullptr;
    return CTQW_OK;
}

ctqw_status ctqw_set_state(ctqw_plan* p, const void* psi, int32_t on_device) {
    if (!p || !psi) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    const int64_t bytes = p->state_off.back() * (p->prob.dtype == CTQW_C128 ? 16 : 8);
    HIP_TRY(p, hipMemcpyAsync(p->psi[0], psi, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              p->stream));
    std::vector<double> ones(p->prob.R, 1.0);
    HIP_TRY(p, hipMemcpyAsync(p->ws + p->lay.scale.off, ones.data(), p->prob.R * 8, hipMemcpyHostToDevice,
                              p->stream));
    HIP_TRY(p, launch_fill_zero(p->ws + p->lay.status.off, 16, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->cur = 0;
    p->steps_done = 0;
    p->have_step_stats = false;
    p->grad_ws = nullptr;
    return CTQW_OK;
}

ctqw_status ctqw_get_state(ctqw_plan* p, void* psi, int32_t on_device) {
    if (!p || !psi) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    if (p->prob.renormalize) {
        RescaleArgs ra{};
        ra.psi = p->psi[p->cur];
        ra.reals = at<RealDev>(p, p->lay.reals);
        ra.scale = at<double>(p, p->lay.scale);
        ra.R = p->prob.R;
        ra.dtype = p->prob.dtype == CTQW_C128 ? 1 : 0;
        HIP_TRY(p, launch_rescale(ra, p->stream));
    }
    const int64_t bytes = p->state_off.back() * (p->prob.dtype == CTQW_C128 ? 16 : 8);
    HIP_TRY(p, hipMemcpyAsync(psi, p->psi[p->cur], bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return CTQW_OK;
}

ctqw_status ctqw_observe(ctqw_plan* p, uint32_t obs, double* out) {
    if (!p || !out) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    if (obs == 0 || (obs & ~p->prob.observables))
        return fail(p, CTQW_ERR_INVALID_ARG, "observables 0x%x not enabled in the problem (0x%x)", obs,
                    p->prob.observables);
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    st = enqueue_observe(p, (obs & CTQW_OBS_PAIR) ? 1 : 0);
    if (st != CTQW_OK) return st;
    return read_snapshot(p, obs, out);
}

ctqw_status ctqw_propagate(ctqw_plan* p, int64_t n_steps, int64_t output_every, uint32_t obs, double* out) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (n_steps < 0 || output_every < 0) return fail(p, CTQW_ERR_INVALID_ARG, "negative step count");
    if (obs & ~p->prob.observables)
        return fail(p, CTQW_ERR_INVALID_ARG, "observables 0x%x not enabled in the problem (0x%x)", obs,
                    p->prob.observables);
    const bool outputs = output_every > 0 && obs != 0;
    if (outputs && !out) return fail(p, CTQW_ERR_INVALID_ARG, "NULL output buffer");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    const int64_t snap = snapshot_len(p, obs);
    const int want_pair = (obs & CTQW_OBS_PAIR) ? 1 : 0;
    int64_t k = 0;
    if (outputs) {
        if ((st = enqueue_observe(p, want_pair)) != CTQW_OK) return st;
        if ((st = read_snapshot(p, obs, out + (k++) * snap)) != CTQW_OK) return st;
    }
    // Steps between outputs form one segment (captured as one graph when
    // use_graph is set); timing collects its events every 256 steps.
    const int64_t seg = outputs ? output_every : (p->timing ? 256 : n_steps);
    for (int64_t s = 0; s < n_steps;) {
        const int64_t n = std::min(seg, n_steps - s);
        if ((st = enqueue_steps(p, n)) != CTQW_OK) return st;
        if (p->timing && (st = collect_timing(p)) != CTQW_OK) return st;
        s += n;
        if (outputs && s % output_every == 0) {
            if ((st = enqueue_observe(p, want_pair)) != CTQW_OK) return st;
            if ((st = read_snapshot(p, obs, out + (k++) * snap)) != CTQW_OK) return st;
        }
    }
    if ((st = collect_timing(p)) != CTQW_OK) return st;
    int32_t status[4];
    if ((st = read_status(p, status)) != CTQW_OK) return st;
    if (status[0] & 2)
        return fail(p, CTQW_ERR_NUMERICAL, "norm alarm or non-finite state in %d realisation-steps", status[1]);
    if (status[0] & 1)
        return fail(p, CTQW_ERR_NOT_CONVERGED, "FP64 truncation test failed in %d realisation-steps", status[1]);
    return CTQW_OK;
}

}  // extern "C"

namespace {

std::string tune_key(ctqw_plan* p) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    const ctqw_problem& pr = p->prob;
    int64_t nsum = 0;
    for (int32_t n : p->N) nsum += n;
    char buf[512];
    snprintf(buf, sizeof buf, "%s|%s|dtype%d|acc%d|m%d|stat%d|bc%d|int%d|R%lld|N%d-%d-%lld|n%d-%d", arch.c_str(),
             ctqw_version(), pr.dtype, pr.dtype == CTQW_C128 ? 1 : pr.accumulation, pr.m, pr.statistics, pr.boundary,
             pr.interaction, (long long)pr.R, *std::min_element(p->N.begin(), p->N.end()), p->max_N,
             (long long)nsum, *std::min_element(p->order.begin(), p->order.end()),
             *std::max_element(p->order.begin(), p->order.end()));
    return buf;
}

bool parse_int_field(const std::string& line, const char* name, int* out) {
    const std::string pat = std::string("\"") + name + "\": ";
    const size_t at = line.find(pat);
    if (at == std::string::npos) return false;
    return sscanf(line.c_str() + at + pat.size(), "%d", out) == 1;
}

bool cache_lookup(const char* path, const std::string& key, ctqw_launch* out, double* ms) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[2048];
    bool found = false;
    const std::string pat = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        std::string s(line);
        if (s.find(pat) == std::string::npos) continue;
        ctqw_launch l{};
        if (parse_int_field(s, "cols_per_lane", &l.cols_per_lane) &&
            parse_int_field(s, "waves_per_block", &l.waves_per_block) &&
            parse_int_field(s, "persistent", &l.persistent) && parse_int_field(s, "waves_per_cu", &l.waves_per_cu)) {
            if (!parse_int_field(s, "chunked", &l.chunked)) l.chunked = 0;
            if (!parse_int_field(s, "band_align", &l.band_align)) l.band_align = 0;
            if (!parse_int_field(s, "terms_per_pass", &l.terms_per_pass)) l.terms_per_pass = 0;
            if (!parse_int_field(s, "band_mode", &l.band_mode)) l.band_mode = 0;
            if (!parse_int_field(s, "row_segments", &l.row_segments)) l.row_segments = 0;
            if (!parse_int_field(s, "three_form", &l.three_form)) l.three_form = 0;
            *out = l;
            const size_t at = s.find("\"ms\": ");
            *ms = at == std::string::npos ? NAN : atof(s.c_str() + at + 6);
            found = true;  // keep the last matching line
        }
    }
    fclose(f);
    return found;
}

void cache_append(const char* path, const std::string& key, const ctqw_launch& l, double ms) {
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f,
            "{\"key\": \"%s\", \"cols_per_lane\": %d, \"waves_per_block\": %d, \"persistent\": %d, "
            "\"waves_per_cu\": %d, \"chunked\": %d, \"band_align\": %d, \"terms_per_pass\": %d, "
            "\"band_mode\": %d, \"row_segments\": %d, \"three_form\": %d, \"ms\": %.6f}\n",
            key.c_str(), l.cols_per_lane, l.waves_per_block, l.persistent, l.waves_per_cu, l.chunked, l.band_align,
            l.terms_per_pass, l.band_mode, l.row_segments, l.three_form, ms);
    fclose(f);
}

// Average step-kernel time of `steps` steps with the current launch shape.
ctqw_status time_steps(ctqw_plan* p, int32_t steps, double* ms) {
    const bool was = p->timing;
    const double t0 = p->timed_ms;
    const int64_t n0 = p->timed_launches;
    ctqw_status st;
    if ((st = enqueue_step(p)) != CTQW_OK) return st;   // warm-up, untimed
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    p->timing = true;
    p->timed_ms = 0.0;
    p->timed_launches = 0;
    for (int32_t s = 0; s < steps; ++s)
        if ((st = enqueue_step(p)) != CTQW_OK) return st;
    if ((st = collect_timing(p)) != CTQW_OK) return st;
    *ms = p->timed_ms / std::max<int64_t>(1, p->timed_launches);
    p->timing = was;
    p->timed_ms = t0;
    p->timed_launches = n0;
    return CTQW_OK;
}

}  // namespace

extern "C" {

ctqw_status ctqw_autotune(ctqw_plan* p, const char* cache_path, int32_t steps, ctqw_launch* best_out,
                          double* best_ms_out) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (steps < 1) return fail(p, CTQW_ERR_INVALID_ARG, "steps must be >= 1");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    const char* path = cache_path ? cache_path : getenv("CTQW_TUNE_CACHE");
    // CTQW_TUNE_TRACE: a file that receives one line per timed candidate
    const char* trace_env = getenv("CTQW_TUNE_TRACE");
    const char* trace = (trace_env && *trace_env) ? trace_env : nullptr;
    const std::string key = tune_key(p);
    const ctqw_launch orig = p->launch;
    ctqw_launch best = orig;
    double best_ms = INFINITY;
    bool cached = false;
    if (path && *path) {
        ctqw_launch l{};
        double ms = NAN;
        if (cache_lookup(path, key, &l, &ms)) {
            l.use_graph = orig.use_graph;
            p->launch = l;
            if (build_tables(p) == CTQW_OK && p->lay.total <= p->ws_bytes) {
                best = l;
                best_ms = ms;
                cached = true;
            }
        }
    }
    if (!cached && p->prob.m == 3) {
        // three particles: terms per pass, the x3 band alignment and the pass form
        for (int form : {0, 1})
        for (int K : {3, 2, 1})
            for (int align : {128, 0}) {
                ctqw_launch c = orig;
                c.terms_per_pass = K;
                c.band_align = align;
                c.three_form = form;
                p->launch = c;
                if (build_tables(p) != CTQW_OK || p->lay.total > p->ws_bytes) continue;
                if ((st = upload_tables(p)) != CTQW_OK) return st;
                double ms = INFINITY;
                if ((st = time_steps(p, steps, &ms)) != CTQW_OK) return st;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        if (!std::isfinite(best_ms)) {
            p->launch = orig;
            build_tables(p);
            return fail(p, CTQW_ERR_UNSUPPORTED, "no launch shape fits the bound workspace");
        }
        if (path && *path) cache_append(path, key, best, best_ms);
    } else if (!cached) {
        for (int mode : {0, 1})
        for (int align : {128, 64, 0})
        for (int chunked : {0, 1})
        for (int P : {1, 2})
            for (int wpb : {1, 2, 4})
                for (int pers : {0, 1})
                    for (int cap : {0, 8, 16}) {
                        if (!pers && cap) continue;
                        if (chunked && (P != 1 || p->prob.m == 3)) continue;   // passes run one column per lane
                        if (mode && (align != 128 || chunked)) continue;        // window-aligned: 128-byte windows
                        ctqw_launch c = orig;
                        c.cols_per_lane = P;
                        c.waves_per_block = wpb;
                        c.persistent = pers;
                        c.waves_per_cu = cap;
                        c.chunked = chunked;
                        c.band_align = align;
                        c.band_mode = mode;
                        p->launch = c;
                        if (build_tables(p) != CTQW_OK || p->lay.total > p->ws_bytes) {
                            if (trace) cache_append(trace, key + " (does not fit the bound workspace)", c, -1.0);
                            continue;
                        }
                        if ((st = upload_tables(p)) != CTQW_OK) return st;
                        double ms = INFINITY;
                        st = time_steps(p, steps, &ms);
                        if (st == CTQW_ERR_UNSUPPORTED) continue;   // block larger than the kernel's bound
                        if (st != CTQW_OK) return st;
                        if (trace) cache_append(trace, key, c, ms);
                        if (ms < best_ms) {
                            best_ms = ms;
                            best = c;
                        }
                    }
        if (!std::isfinite(best_ms)) {
            p->launch = orig;
            build_tables(p);
            return fail(p, CTQW_ERR_UNSUPPORTED, "no launch shape fits the bound workspace");
        }
        // the row split of the best shape: caps other than the default's
        if (p->prob.m == 2 && !best.chunked) {
            int64_t n_auto = -1;
            p->launch = best;
            if (build_tables(p) == CTQW_OK) n_auto = (int64_t)p->items.size();
            for (int seg : {1, 2, 4, 8}) {
                ctqw_launch c = best;
                c.row_segments = seg;
                p->launch = c;
                if (build_tables(p) != CTQW_OK || p->lay.total > p->ws_bytes) continue;
                if ((int64_t)p->items.size() == n_auto) continue;   // the same partition as the default
                if ((st = upload_tables(p)) != CTQW_OK) return st;
                double ms = INFINITY;
                st = time_steps(p, steps, &ms);
                if (st == CTQW_ERR_UNSUPPORTED) continue;
                if (st != CTQW_OK) return st;
                if (trace) cache_append(trace, key, c, ms);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        }
        if (path && *path) cache_append(path, key, best, best_ms);
    }
    p->launch = best;
    if ((st = build_tables(p)) != CTQW_OK) return st;
    if ((st = upload_tables(p)) != CTQW_OK) return st;
    p->have_step_stats = false;
    if (best_out) *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return CTQW_OK;
}

}  // extern "C"

namespace {

// Gradient workspace: checkpoints, recomputed segment states, the Taylor
// vectors v_1..v_{n-1} of one step, two Horner vectors, two adjoint states,
// then FP64 accumulators.
struct GradLayout {
    int64_t S = 0, n_ckpt = 0, n_seg = 0, n_v = 0;
    int64_t ckpt = 0, seg = 0, v = 0, u = 0, lam = 0;
    int64_t gJ = 0, gE = 0, gV = 0, gR = 0, row_loss = 0, site_w = 0, out = 0;
    int nb = 1;
    int64_t total = 0;
};

GradLayout grad_layout(const ctqw_plan* p, int64_t n_steps, int64_t C) {
    GradLayout g;
    const int64_t esz = p->prob.dtype == CTQW_C128 ? 16 : 8;
    g.S = (p->state_off.back() * esz + 255) & ~int64_t(255);
    g.n_ckpt = n_steps > 0 ? (n_steps + C - 1) / C : 1;
    g.n_seg = std::max<int64_t>(0, std::min(C, std::max<int64_t>(n_steps, 1)) - 1);
    g.n_v = std::max(0, p->levels - 1);
    int64_t o = 0;
    g.ckpt = o; o += g.n_ckpt * g.S;
    g.seg = o; o += g.n_seg * g.S;
    g.v = o; o += g.n_v * g.S;
    g.u = o; o += 2 * g.S;
    g.lam = o; o += 2 * g.S;
    auto dbl = [&](int64_t n) { const int64_t r = o; o += (n * 8 + 255) & ~int64_t(255); return r; };
    g.gJ = dbl(p->site_total);
    g.gE = dbl(p->site_total);
    // row parts of the backward passes: one partial per band and row (the
    // Horner passes' narrowest bands)
    const int hw = pipe_band_width(pipe_max_levels(p->prob.dtype == CTQW_C128 ? 1 : 0, true));
    g.nb = std::max(1, (p->max_N + hw - 1) / hw);
    g.gV = dbl((int64_t)p->prob.R * g.nb * p->max_N);
    g.gR = dbl((int64_t)p->prob.R * g.nb * p->max_N);
    g.row_loss = dbl(p->site_total);
    g.site_w = dbl(p->max_N);
    g.out = dbl(2 * (int64_t)p->max_N + 1);
    g.total = o;
    return g;
}

double inv_fact(int j) {
    double f = 1.0;
    for (int k = 2; k <= j; ++k) f *= k;
    return 1.0 / f;
}

}  // namespace

extern "C" {

ctqw_status ctqw_gradient_workspace(const ctqw_plan* p, int64_t n_steps, int64_t ckpt_every, int64_t* bytes) {
    if (!p || !bytes) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_INVALID_ARG, "NULL argument");
    if (!p->params_set) return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_STATE, "parameters not set");
    if (n_steps < 0 || ckpt_every < 1)
        return fail(const_cast<ctqw_plan*>(p), CTQW_ERR_INVALID_ARG, "need n_steps >= 0 and ckpt_every >= 1");
    *bytes = grad_layout(p, n_steps, ckpt_every).total;
    return CTQW_OK;
}

ctqw_status ctqw_forward_ckpt(ctqw_plan* p, int64_t n_steps, int64_t ckpt_every, void* gws, int64_t gws_bytes) {
    if (p && p->tele_amp > 0.0)
        return fail(p, CTQW_ERR_UNSUPPORTED, "gradients are built for static noise (switching noise is on)");
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!gws) return fail(p, CTQW_ERR_INVALID_ARG, "NULL gradient workspace");
    if (n_steps < 0 || ckpt_every < 1) return fail(p, CTQW_ERR_INVALID_ARG, "need n_steps >= 0 and ckpt_every >= 1");
    if (p->prob.renormalize) return fail(p, CTQW_ERR_UNSUPPORTED, "gradients need renormalize == 0 (a linear map)");
    if (p->group_N.size() != 1)
        return fail(p, CTQW_ERR_UNSUPPORTED, "gradients with respect to shared baselines need one lattice size");
    if (p->prob.m == 3) return fail(p, CTQW_ERR_UNSUPPORTED, "gradients are built for one and two particles");
    if (p->prob.m == 2 && p->prob.statistics == CTQW_FERMION)
        return fail(p, CTQW_ERR_UNSUPPORTED, "gradients are built for distinguishable particles and bosons");
    {
        // the adjoint passes address a realisation's amplitudes through one
        // buffer resource, whose length is a 31-bit byte count
        const int64_t amps = p->prob.m == 1 ? (int64_t)p->max_N : (int64_t)p->max_N * p->max_N;
        if (amps * (p->prob.dtype == CTQW_C128 ? 16 : 8) > INT32_MAX)
            return fail(p, CTQW_ERR_UNSUPPORTED, "gradients need each realisation's state under 2 GiB (N = %d)",
                        p->max_N);
    }
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    const GradLayout g = grad_layout(p, n_steps, ckpt_every);
    if (gws_bytes < g.total)
        return fail(p, CTQW_ERR_INVALID_ARG, "gradient workspace too small (%lld < %lld bytes)", (long long)gws_bytes,
                    (long long)g.total);
    if (reinterpret_cast<uintptr_t>(gws) & 255) return fail(p, CTQW_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    uint8_t* G = static_cast<uint8_t*>(gws);
    hipStream_t s = p->stream;
    const int64_t bytes = p->state_off.back() * (p->prob.dtype == CTQW_C128 ? 16 : 8);
    const int64_t C = ckpt_every;
    // forward, keeping the state at steps 0, C, 2C, ...; every realisation
    // runs the batch's largest order, the polynomial the adjoint inverts
    p->one_depth = true;
    for (int64_t k = 0; k < n_steps; ++k) {
        if (k % C == 0)
            HIP_TRY(p, hipMemcpyAsync(G + g.ckpt + (k / C) * g.S, p->psi[p->cur], bytes, hipMemcpyDeviceToDevice, s));
        if ((st = enqueue_step(p)) != CTQW_OK) {
            p->one_depth = false;
            return st;
        }
    }
    p->one_depth = false;
    if (n_steps == 0) HIP_TRY(p, hipMemcpyAsync(G + g.ckpt, p->psi[p->cur], bytes, hipMemcpyDeviceToDevice, s));
    p->grad_ws = gws;
    p->grad_steps = n_steps;
    p->grad_ckpt = ckpt_every;
    p->grad_tables = p->table_version;
    return CTQW_OK;
}

ctqw_status ctqw_backward(ctqw_plan* p, int32_t kind, const double* site_w, void* gws, int64_t gws_bytes,
                          double* loss, double* grad_J, double* grad_eps) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!site_w || !gws || !loss || !grad_J || !grad_eps) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    if (kind != CTQW_LOSS_ONE_BODY && kind != CTQW_LOSS_PRODUCT)
        return fail(p, CTQW_ERR_INVALID_ARG, "unknown loss kind %d", kind);
    if (gws != p->grad_ws || p->grad_tables != p->table_version)
        return fail(p, CTQW_ERR_STATE, "no ctqw_forward_ckpt with this workspace since the last change");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    const int64_t n_steps = p->grad_steps;
    const int64_t ckpt_every = p->grad_ckpt;
    const GradLayout g = grad_layout(p, n_steps, ckpt_every);
    if (gws_bytes < g.total)
        return fail(p, CTQW_ERR_INVALID_ARG, "gradient workspace too small (%lld < %lld bytes)", (long long)gws_bytes,
                    (long long)g.total);
    for (int i = 0; i < p->N[0]; ++i)
        if (!is_fin(site_w[i])) return fail(p, CTQW_ERR_INVALID_ARG, "site weight %d is not finite", i);
    p->grad_ws = nullptr;   // one backward per forward

    uint8_t* G = static_cast<uint8_t*>(gws);
    hipStream_t s = p->stream;
    const ctqw_problem& pr = p->prob;
    const int n = p->levels;
    const int N = p->N[0];
    const int rows = pr.m == 1 ? 1 : N;
    const int dtype = pr.dtype == CTQW_C128 ? 1 : 0;
    const int64_t C = ckpt_every;
    auto state = [&](int64_t off, int64_t k) { return static_cast<void*>(G + off + k * g.S); };

    HIP_TRY(p, launch_fill_zero(G + g.gJ, g.site_w - g.gJ, s));
    HIP_TRY(p, hipMemcpyAsync(G + g.site_w, site_w, N * 8, hipMemcpyHostToDevice, s));

    const RealDev* reals = at<RealDev>(p, p->lay.reals);
    const int64_t* site_off = at<int64_t>(p, p->lay.site_off);
    AdjWeightArgs wa{};
    wa.psi = p->psi[p->cur];
    wa.lam = state(g.lam, 0);
    wa.reals = reals;
    wa.site_off = site_off;
    wa.site_w = reinterpret_cast<const double*>(G + g.site_w);
    wa.row_loss = reinterpret_cast<double*>(G + g.row_loss);
    wa.inv_R = 1.0 / (double)pr.R;
    wa.kind = kind;
    wa.R = pr.R;
    wa.max_rows = rows;
    wa.dtype = dtype;
    HIP_TRY(p, launch_adj_weights(wa, s));

    // K levels per pass (adjoint_pipe.hpp): forward vectors and Horner levels
    AdjPipeArgs pa{};
    pa.reals = reals;
    pa.Jt = dtype ? static_cast<const void*>(at<double>(p, p->lay.Jd)) : static_cast<const void*>(at<float>(p, p->lay.Jf));
    pa.Et = dtype ? static_cast<const void*>(at<double>(p, p->lay.Ed)) : static_cast<const void*>(at<float>(p, p->lay.Ef));
    pa.dt = pr.dt;
    pa.site_off = site_off;
    pa.gJ = reinterpret_cast<double*>(G + g.gJ);
    pa.gE = reinterpret_cast<double*>(G + g.gE);
    pa.gV = reinterpret_cast<double*>(G + g.gV);
    pa.gR = reinterpret_cast<double*>(G + g.gR);
    pa.R = pr.R;
    pa.nb = g.nb;
    pa.max_n = p->max_N;
    pa.row_stride = p->max_N;
    pa.dtype = dtype;
    pa.periodic = pr.boundary == CTQW_PERIODIC ? 1 : 0;
    pa.layout = pr.m == 1 ? 0 : (pr.statistics == CTQW_DISTINGUISHABLE ? 1 : 2);
    const int kf = pipe_max_levels(dtype, false), kh = pipe_max_levels(dtype, true);
    // passes of at most kmax levels, as even as the count allows
    auto pass_levels = [](int left, int kmax) {
        const int passes = (left + kmax - 1) / kmax;
        return (left + passes - 1) / passes;
    };

    int lc = 0;   // state(g.lam, lc) holds lambda_{k+1}
    std::vector<const void*> segp(C), vp(n);
    for (int64_t sg = g.n_ckpt - 1; sg >= 0 && n_steps > 0; --sg) {
        const int64_t k0 = sg * C;
        const int64_t len = std::min(C, n_steps - k0);
        segp[0] = state(g.ckpt, sg);
        for (int64_t k = 1; k < len; ++k) {
            segp[k] = state(g.seg, k - 1);
            if ((st = enqueue_step_io(p, segp[k - 1], const_cast<void*>(segp[k]))) != CTQW_OK) return st;
        }
        for (int64_t k = len - 1; k >= 0; --k) {
            const void* lam = state(g.lam, lc);
            // v_i = A^i psi_k, K levels per pass, every level stored
            vp[0] = segp[k];
            for (int i = 1; i < n; ++i) vp[i] = state(g.v, i - 1);
            for (int i0 = 0; i0 < n - 1;) {
                const int K = pass_levels(n - 1 - i0, kf);
                AdjPipeArgs a = pa;
                a.x = vp[i0];
                a.xs = 1.0;
                a.sign = +1;
                a.levels = K;
                for (int l = 1; l <= K; ++l) a.y[l - 1] = const_cast<void*>(vp[i0 + l]);
                HIP_TRY(p, launch_adj_pipe(a, s));
                i0 += K;
            }
            // Horner: level L contracts u_L with v_L and forms u_{L-1} = lambda / L! + A^dagger u_L
            // (lambda_k at L = 0); u_{n-1} = lambda / n! is the first pass's scaled input.  A pass
            // of K levels runs L = Lhi .. Lhi - K + 1 and stores only its last level.
            int uc = 0;
            const void* u = lam;
            double us = inv_fact(n);
            for (int Lhi = n - 1; Lhi >= 0;) {
                const int K = pass_levels(Lhi + 1, kh);
                void* y = Lhi - K + 1 > 0 ? state(g.u, uc) : state(g.lam, 1 - lc);
                AdjPipeArgs a = pa;
                a.x = u;
                a.xs = us;
                a.z = lam;
                a.sign = -1;
                a.levels = K;
                a.contract = 1;
                for (int l = 1; l <= K; ++l) {
                    a.v[l - 1] = vp[Lhi - l + 1];
                    a.cz[l] = inv_fact(Lhi - l + 1);
                }
                a.y[K - 1] = y;
                HIP_TRY(p, launch_adj_pipe(a, s));
                u = y;
                us = 1.0;
                uc ^= 1;
                Lhi -= K;
            }
            lc ^= 1;
        }
    }

    AdjReduceArgs ra{};
    ra.gJ = pa.gJ;
    ra.gE = pa.gE;
    ra.gV = pa.gV;
    ra.gR = pa.gR;
    ra.nb = g.nb;
    ra.row_stride = p->max_N;
    ra.row_loss = wa.row_loss;
    ra.site_off = site_off;
    ra.out = reinterpret_cast<double*>(G + g.out);
    ra.R = pr.R;
    ra.N = N;
    ra.rows = rows;
    ra.dt = pr.dt;
    HIP_TRY(p, launch_adj_reduce(ra, s));
    std::vector<double> host(2 * (size_t)N + 1);
    HIP_TRY(p, hipMemcpyAsync(host.data(), G + g.out, host.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(p, hipStreamSynchronize(s));
    const int nb = n_bonds(pr, N);
    std::memcpy(grad_J, host.data(), nb * 8);
    std::memcpy(grad_eps, host.data() + N, N * 8);
    *loss = host[2 * N];
    return CTQW_OK;
}

ctqw_status ctqw_loss(ctqw_plan* p, int32_t kind, const double* site_w, void* gws, int64_t gws_bytes, double* loss) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!site_w || !gws || !loss) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    if (kind != CTQW_LOSS_ONE_BODY && kind != CTQW_LOSS_PRODUCT)
        return fail(p, CTQW_ERR_INVALID_ARG, "unknown loss kind %d", kind);
    if (p->group_N.size() != 1) return fail(p, CTQW_ERR_UNSUPPORTED, "the loss needs one lattice size");
    if (p->prob.m == 3) return fail(p, CTQW_ERR_UNSUPPORTED, "the loss is built for one and two particles");
    if (p->prob.m == 2 && p->prob.statistics == CTQW_FERMION)
        return fail(p, CTQW_ERR_UNSUPPORTED, "the loss is built for distinguishable particles and bosons");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    const GradLayout g = grad_layout(p, 0, 1);
    if (gws_bytes < g.total)
        return fail(p, CTQW_ERR_INVALID_ARG, "workspace too small (%lld < %lld bytes)", (long long)gws_bytes,
                    (long long)g.total);
    if (reinterpret_cast<uintptr_t>(gws) & 255) return fail(p, CTQW_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const int N = p->N[0];
    for (int i = 0; i < N; ++i)
        if (!is_fin(site_w[i])) return fail(p, CTQW_ERR_INVALID_ARG, "site weight %d is not finite", i);
    // Scratch regions of a zero-step gradient layout at the end of the
    // workspace, so that checkpoints of a pending forward run survive.
    uint8_t* G = static_cast<uint8_t*>(gws) + (gws_bytes - g.total) / 256 * 256;
    hipStream_t s = p->stream;
    const ctqw_problem& pr = p->prob;
    const int rows = pr.m == 1 ? 1 : N;
    HIP_TRY(p, launch_fill_zero(G + g.gJ, g.site_w - g.gJ, s));
    HIP_TRY(p, hipMemcpyAsync(G + g.site_w, site_w, N * 8, hipMemcpyHostToDevice, s));
    AdjWeightArgs wa{};
    wa.psi = p->psi[p->cur];
    wa.lam = G + g.lam;
    wa.reals = at<RealDev>(p, p->lay.reals);
    wa.site_off = at<int64_t>(p, p->lay.site_off);
    wa.site_w = reinterpret_cast<const double*>(G + g.site_w);
    wa.row_loss = reinterpret_cast<double*>(G + g.row_loss);
    wa.inv_R = 1.0 / (double)pr.R;
    wa.kind = kind;
    wa.R = pr.R;
    wa.max_rows = rows;
    wa.dtype = pr.dtype == CTQW_C128 ? 1 : 0;
    HIP_TRY(p, launch_adj_weights(wa, s));
    AdjReduceArgs ra{};
    ra.gJ = reinterpret_cast<const double*>(G + g.gJ);
    ra.gE = reinterpret_cast<const double*>(G + g.gE);
    ra.gV = reinterpret_cast<const double*>(G + g.gV);
    ra.gR = reinterpret_cast<const double*>(G + g.gR);
    ra.nb = g.nb;
    ra.row_stride = p->max_N;
    ra.row_loss = wa.row_loss;
    ra.site_off = wa.site_off;
    ra.out = reinterpret_cast<double*>(G + g.out);
    ra.R = pr.R;
    ra.N = N;
    ra.rows = rows;
    ra.dt = pr.dt;
    HIP_TRY(p, launch_adj_reduce(ra, s));
    HIP_TRY(p, hipMemcpyAsync(loss, G + g.out + 2 * (int64_t)N * 8, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(p, hipStreamSynchronize(s));
    return CTQW_OK;
}

ctqw_status ctqw_gradient(ctqw_plan* p, int64_t n_steps, int64_t ckpt_every, int32_t kind, const double* site_w,
                          void* gws, int64_t gws_bytes, double* loss, double* grad_J, double* grad_eps) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (!site_w || !loss || !grad_J || !grad_eps) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    if (kind != CTQW_LOSS_ONE_BODY && kind != CTQW_LOSS_PRODUCT)
        return fail(p, CTQW_ERR_INVALID_ARG, "unknown loss kind %d", kind);
    ctqw_status st = ctqw_forward_ckpt(p, n_steps, ckpt_every, gws, gws_bytes);
    if (st != CTQW_OK) return st;
    return ctqw_backward(p, kind, site_w, gws, gws_bytes, loss, grad_J, grad_eps);
}

ctqw_status ctqw_set_timing(ctqw_plan* p, int32_t enable) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (p->bound) {
        ctqw_status st = collect_timing(p);
        if (st != CTQW_OK) return st;
    }
    p->timing = enable != 0;
    p->timed_ms = 0.0;
    p->timed_launches = 0;
    return CTQW_OK;
}

ctqw_status ctqw_get_timing(ctqw_plan* p, double* ms, int64_t* launches) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    if (p->bound) {
        ctqw_status st = collect_timing(p);
        if (st != CTQW_OK) return st;
    }
    if (ms) *ms = p->timed_ms;
    if (launches) *launches = p->timed_launches;
    return CTQW_OK;
}

ctqw_status ctqw_realization_norms(ctqw_plan* p, double* norm2, double* tail2) {
    if (!p) return fail(nullptr, CTQW_ERR_INVALID_ARG, "NULL plan");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    if (!p->have_step_stats) return fail(p, CTQW_ERR_STATE, "no step taken yet");
    if (norm2) HIP_TRY(p, hipMemcpyAsync(norm2, p->ws + p->lay.norm2.off, p->prob.R * 8, hipMemcpyDeviceToHost, p->stream));
    if (tail2) HIP_TRY(p, hipMemcpyAsync(tail2, p->ws + p->lay.tail2.off, p->prob.R * 8, hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(p, hipStreamSynchronize(p->stream));
    return CTQW_OK;
}

ctqw_status ctqw_stats(ctqw_plan* p, ctqw_step_stats* out) {
    if (!p || !out) return fail(p, CTQW_ERR_INVALID_ARG, "NULL argument");
    ctqw_status st = ensure_ready(p);
    if (st != CTQW_OK) return st;
    std::memset(out, 0, sizeof *out);
    out->steps_done = p->steps_done;
    out->min_order = *std::min_element(p->order.begin(), p->order.end());
    out->max_order = *std::max_element(p->order.begin(), p->order.end());
    int32_t status[4];
    if ((st = read_status(p, status)) != CTQW_OK) return st;
    out->flags = status[0];
    out->alarms = status[1];
    if (!p->have_step_stats) {
        out->min_norm = out->max_norm = NAN;
        out->max_tail_ratio = NAN;
        return CTQW_OK;
    }
    std::vector<double> n2(p->prob.R), t2(p->prob.R);
    if ((st = ctqw_realization_norms(p, n2.data(), t2.data())) != CTQW_OK) return st;
    double mn = INFINITY, mx = -INFINITY, tr = 0.0;
    const double tol = p->prob.taylor_tol;
    for (int64_t r = 0; r < p->prob.R; ++r) {
        const double nr = std::sqrt(n2[r]);
        mn = std::min(mn, nr);
        mx = std::max(mx, nr);
        if (tol > 0) tr = std::max(tr, std::sqrt(t2[r]) / (tol * nr));
    }
    out->min_norm = mn;
    out->max_norm = mx;
    out->max_tail_ratio = tol > 0 ? tr : NAN;
    return CTQW_OK;
}

}  // extern "C"
