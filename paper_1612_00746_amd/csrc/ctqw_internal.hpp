// Internal tables and launch descriptors shared by the host runtime and the
// HIP kernels of libctqw.  Not part of the public ABI (include/ctqw.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ctqw {

// Bits of RealDev::flags.
enum : int32_t {
    RF_PERIODIC = 1,   // ring: bond N-1 joins node N-1 and node 0
    RF_TRIANGLE = 2,   // two bosons or fermions stored as the upper triangle x1 <= x2
    RF_NEAREST = 4,    // interaction on pairs at chain distance 1
    RF_FERMION = 8,    // triangle of two fermions: the diagonal x1 == x2 is held at 0
    RF_NO_EPS = 16,    // all on-site energies are 0: the diagonal of H is the interaction alone
};

// One realisation, as the kernels see it.  The walk of m = 1 or 2 particles
// is a grid of `rows` x N amplitudes: rows = N for two particles (x1 runs
// over rows, x2 over columns) and rows = 1 for one particle.
struct RealDev {
    int64_t state_off;   // first amplitude in a state buffer
    int32_t N;           // nodes (columns)
    int32_t rows;        // rows of the amplitude grid (1 or N)
    int32_t order;       // Taylor terms per step
    int32_t param_off;   // J / eps of this realisation: [N] each, J padded
    int32_t row_param_off;  // J / eps for the row axis (a zero block if rows == 1)
    int32_t flags;       // RF_*
    double U;            // interaction strength (0 for one particle)
    double tail_factor;  // remainder estimate / ||Phi^(n)||, n = the realisation's order
    double tail_factor_max;  // the same for the batch's largest order (one-depth launches)
};

// One work item: a band of columns of one realisation, swept over all rows.
// The wave holds columns [w0, w0 + 64 * P); only [lo, hi) are written, the
// rest is halo that is recomputed by the neighbouring band.
struct ItemDev {
    int32_t real;
    int32_t w0;          // first window column (negative allowed on a ring)
    int32_t lo, hi;      // output columns
    int32_t row0;        // first swept row (negative allowed on a ring)
    int32_t nrows;       // swept rows
    int32_t out_lo, out_hi;  // output rows (absolute)
};

// Persistent step launches claim work from one list per XCD: the hardware
// hands a grid's blocks to the eight XCDs of the device in turn (block b to
// XCD b mod 8), and each XCD has its own L2, so the bands that share halo
// columns are listed together on one XCD.  A block whose list is empty
// takes work from the next lists.
constexpr int kClaimLists = 8;

struct StepArgs {
    const void* psi_in;
    void* psi_out;
    const RealDev* reals;
    const ItemDev* items;
    const int32_t* item_order;   // processing order (largest first)
    int32_t* claim;              // persistent launch: kClaimLists counters, zero at launch
    const int32_t* list_off;     // persistent launch: kClaimLists + 1 offsets into
                                 // item_order; list x = [list_off[x], list_off[x + 1])
    int32_t n_items;
    int32_t n_waves;             // persistent launch: waves in the grid
    const double* Jd;
    const double* Ed;
    const float* Jf;
    const float* Ef;
    const double* scale;         // [R] factor applied when loading the state
    double* norm_part;           // [n_items] sum of w |psi_out|^2 of each item
    double* tail_part;           // [n_items] sum of w |Phi^(n)|^2 of each item
    double dt;
    int32_t persistent;          // 1: grid of n_waves waves claiming items
    // Chunked step (orders above the fused depth): one pass of the kernel's
    // depth NT continues the series from Psi_s (psi_in, true complex values)
    // and the partial sum acc_in, writing the new partial sum to psi_out and
    // Psi_{s+NT} to seed_out.  Unused by the fused kernel.
    const void* acc_in;
    void* seed_out;              // null on the last pass
    double coef[16];             // 1/(s+j)! for j = 1..NT, 0 past the order
    double tail_coef;            // 1/n! (last pass)
    int32_t tail_level;          // level of the order's last term (last pass), else 0
    int32_t first;               // first pass: loads carry the realisation's scale
    int32_t last;                // last pass: norm and tail partials
};

struct StepConfig {
    int dtype;          // 0: complex64, 1: complex128
    int kahan;          // compensated accumulation (complex64 only)
    int triangle;       // two bosons in the upper-triangle layout
    int cols_per_lane;  // 1 or 2
    int levels;         // compiled pipeline depth (>= max order in the batch)
    int waves_per_block;
    int persistent;
    int grid_blocks;    // persistent: blocks to launch
    int vec;            // complex64, two columns per lane: paired 16-byte accesses
    int two;            // complex64 full grid: items of orders levels and levels - 1
};

// Host entry points implemented in the .hip translation units.
hipError_t launch_step(const StepConfig& cfg, const StepArgs& args, hipStream_t stream);
// Chunked passes: terms per pass (8 for complex64, 4 for complex128, whose
// pipeline at depth 8 needs more than 256 VGPRs), launched like the fused
// kernel (cfg.levels is ignored, cols_per_lane must be 1).
constexpr int chunk_depth(int dtype) { return dtype == 1 ? 4 : 8; }
hipError_t launch_chunk_pass(const StepConfig& cfg, const StepArgs& args, hipStream_t stream);
hipError_t chunk_occupancy(const StepConfig& cfg, int* blocks_per_cu);
hipError_t chunk_max_block(const StepConfig& cfg, int* threads);
// Smallest compiled pipeline depth >= order (-1 if none).
int step_levels_bucket(int dtype, int cols_per_lane, int order);
hipError_t step_occupancy(const StepConfig& cfg, int* blocks_per_cu);
// Largest block the selected kernel was compiled for (its launch bound).
hipError_t step_max_block(const StepConfig& cfg, int* threads);

struct FinalizeArgs {
    const int32_t* item_first;   // [R + 1] home items of each realisation
    const double* norm_part;
    const double* tail_part;
    const RealDev* reals;
    double* norm2;               // [R]
    double* tail2;               // [R] estimated squared truncation error
    double* scale;               // [R] next load scale
    int32_t* status;             // [4]: flags, alarm count lo, alarm count hi, pad
    int64_t R;
    double tol2;
    double norm_alarm;
    int renormalize;
    int use_max;                 // the step ran every realisation at the batch's largest order
};
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t stream);

struct InitArgs {
    void* psi;
    const RealDev* reals;
    const int32_t* sites;        // [m] or [R*m]
    int32_t per_real;
    int32_t m;
    int64_t R;
    int64_t total;               // amplitudes
    int dtype;
};
hipError_t launch_init(const InitArgs& a, hipStream_t stream);

struct ObsArgs {
    const void* psi;
    const RealDev* reals;
    const double* scale;
    double* colsum;              // [sum_r N_r]
    double* rowsum;              // [sum_r N_r]
    double* diag;                // [sum_r N_r] p(i, i) (two particles)
    const int64_t* site_off;     // [R] offsets into the per-site arrays
    const int32_t* group_members;  // realisations ordered by group
    const int32_t* group_first;  // [G + 1]
    const int32_t* group_N;      // [G]
    const int64_t* group_out;    // [G] offset of the group's block in out
    double* out;                 // device snapshot buffer
    int64_t R;
    int32_t G;
    int32_t m;
    int32_t max_N;
    int32_t want_pair;
    int dtype;
};
hipError_t launch_observables(const ObsArgs& a, hipStream_t stream);

struct RescaleArgs {
    void* psi;
    const RealDev* reals;
    double* scale;
    int64_t R;
    int dtype;
};
hipError_t launch_rescale(const RescaleArgs& a, hipStream_t stream);

hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t stream);

// ------------------------------------------------------- three particles
// Three particles, K terms chained per pass: one work item is a tile of the
// (x2, x3) plane swept over the x1 planes.  The tile's window is 64 x3
// columns from z0 and (rows per block) x2 rows from y0 (either may start
// below 0 on a ring); only [zlo, zhi) x [ylo, yhi) is written, the rest is
// halo that the neighbouring tiles write.
struct Item3Dev {
    int32_t real;
    int32_t z0, zlo, zhi;
    int32_t y0, ylo, yhi;
    int32_t x0;              // first swept plane (-K on a ring)
    int32_t nplanes;         // swept planes
    int32_t plane_lo, plane_hi;   // output planes (absolute)
    int32_t pad;
};

// One pass of K levels: X = Psi_s (psi, scaled by the load scale, on the
// first pass), base = the partial sum before the pass (psi on the first);
// writes the partial sum after it (the new state on the last pass) and
// Psi_{s+K} (before the last pass).
struct Step3cArgs {
    const void* x_in;
    const void* base_in;
    void* sum_out;
    void* seed_out;          // null on the last pass
    const RealDev* reals;
    const Item3Dev* items;
    const void* Jt;          // dt-scaled tables (dtype of the state)
    const void* Et;
    const double* scale;
    double* norm_part;       // [n_items] (last pass)
    double* tail_part;
    double dt;
    double coef[4];          // 1/(s+j)! for j = 1..K, 0 past the order
    double tail_coef;        // 1/n!
    int32_t tail_level;      // level of the order's last term (last pass), else 0
    int32_t first;
    int32_t last;
    int32_t n_items;
};
// Terms per pass of the compiled three-particle kernels: 1..3.  Rows of the
// x2 window of one block for a (dtype, K), 0 if not compiled.
int step3c_rows_per_block(int dtype, int K);
hipError_t launch_step3c(const Step3cArgs& a, int dtype, int K, hipStream_t stream);

struct Obs3Args {
    const void* psi;
    const RealDev* reals;
    const double* scale;
    double* M;               // [R][3][N][N] two-body marginals
    double* occ_terms;       // [G][N][N]
    const int32_t* group_members;
    const int32_t* group_first;
    const int32_t* group_N;
    const int64_t* group_out;
    double* out;
    int64_t R;
    int32_t G;
    int32_t max_N;
    int32_t want_pair;
};
hipError_t launch_obs3(const Obs3Args& a, int dtype, hipStream_t stream);

// ---------------------------------------------------------------- adjoint
// Backward passes: a block of kSweepSegs waves splits a band's rows into
// consecutive segments, one wave each.
constexpr int kSweepSegs = 4;

struct AdjWeightArgs {
    const void* psi;
    void* lam;
    const RealDev* reals;
    const int64_t* site_off;
    const double* site_w;
    double* row_loss;
    double inv_R;
    int kind;            // 0: one-body sum, 1: product
    int64_t R;
    int max_rows;
    int dtype;
};
hipError_t launch_adj_weights(const AdjWeightArgs& a, hipStream_t stream);

struct AdjReduceArgs {
    const double* gJ;
    const double* gE;
    const double* gV;
    const double* gR;
    int nb;
    int row_stride;
    const double* row_loss;
    const int64_t* site_off;
    double* out;         // [2N + 1]: dL/dJ, dL/deps, loss
    int64_t R;
    int N;
    int rows;
    double dt;
};
hipError_t launch_adj_reduce(const AdjReduceArgs& a, hipStream_t stream);

}  // namespace ctqw

namespace ctqw {
// One particle on a two-dimensional lattice (lattice.hip).
constexpr int kLatticeMaxOrderC64 = 12;
constexpr int kLatticeMaxOrderC128 = 10;
struct LatticeArgs {
    const void* Jx;          // [R][Ly][Lx] bond to (x + 1, y), the state's real type
    const void* Jy;          // [R][Ly][Lx] bond to (x, y + 1)
    const void* eps;         // [R][Ly][Lx] on-site energies
    void* tab;               // dt-scaled tables: right bonds, bonds below, energies ([3][R][Ly][Lx])
    const void* psi_in;      // [R][Ly][Lx]
    void* psi_out;
    double* norm_part;       // [R][nb] squared FP64 norm of each item's output
    int32_t Lx, Ly, R, px, py, nb, n_items;
    double dt;
};
int lattice_max_order(int dtype);
hipError_t launch_lattice_scale(const LatticeArgs& a, int dtype, hipStream_t stream);
hipError_t launch_lattice_step(const LatticeArgs& a, int dtype, int order, hipStream_t stream);
hipError_t launch_lattice_norms(const double* part, int32_t nb, int32_t R, double* out, hipStream_t stream);
}  // namespace ctqw

namespace ctqw {
// Record the message returned by ctqw_last_error(NULL) and return status.
int report_error(int status, const char* message);
}  // namespace ctqw
