// Pipelined passes of the discrete adjoint (the kernels that replace one
// sweep per level by one sweep per K levels).
//
// A pass applies K levels of
//     Y_l = cz_l Z + s (-i) (dt H) Y_(l-1),   Y_0 = xs X,   l = 1 .. K,
// in one sweep down the rows, the levels chained in registers as in the
// forward step: at sweep step i row i of X (and Z) enters, level l forms
// row i - l of Y_l from level l - 1's rows i - l - 1, i - l, i - l + 1, and
// row i - K of the last level is complete.  Optionally every level's rows
// are stored (y[l - 1]), and level l contracts its input Y_(l-1) with v[l - 1]
// (Im <Y_(l-1)| E |v> for every bond and site operator E, the sums of the
// one-level sweep).  The backward step of the adjoint is then
//   * the forward vectors v_1 .. v_(n-1) = A^i psi_k: passes with s = +1, no
//     Z, every level stored;
//   * the Horner chain u_(L-1) = lambda / L! + A^dagger u_L, contracted with
//     v_L at every level (u_(n-1) = lambda / n!, the first pass's scaled
//     input; lambda_k at L = 0): passes with s = -1, Z = lambda, the last
//     level stored,
// reading each vector once per pass instead of once per level.
//
// Work item: a band of 64 - 2K output columns of one realisation, held by
// one wave with K halo columns on either side (level l is exact up to l
// columns from the window's edges, and the contraction reaches one column
// further), swept down the rows in kSweepSegs row segments (one wave each)
// that start K rows before their first output row and end K rows after the
// last (open chains: clamped to the grid, whose outside is zero).
#pragma once

#include "ctqw_internal.hpp"

namespace ctqw {

// Levels per pass compiled for each state type: forward-vector passes, and
// Horner passes (whose contraction holds two more rows per level, and more
// would spill at two waves per SIMD).
constexpr int kPipeMaxLevelsC64 = 8;
constexpr int kPipeMaxLevelsC128 = 4;
constexpr int kPipeMaxHornerC64 = 3;
constexpr int kPipeMaxHornerC128 = 2;
constexpr int kPipeMaxLevels = 8;

struct AdjPipeArgs {
    const void* x;                      // level 0 input (never null)
    double xs;                          // its scale: Y_0 = xs X
    const void* z;                      // source of every level (may be null)
    double cz[kPipeMaxLevels + 1];      // cz[l]: weight of Z in level l (1 .. K)
    int sign;                           // +1: A = -i dt H; -1: A^dagger
    void* y[kPipeMaxLevels];            // y[l - 1]: where level l is stored (null: not stored)
    const void* v[kPipeMaxLevels];      // v[l - 1]: contraction partner of level l's input
    const RealDev* reals;
    const void* Jt;                     // dt-scaled tables of the step kernel (dtype of the state)
    const void* Et;
    double dt;
    const int64_t* site_off;
    double* gJ;                         // column parts per realisation (bond b / site b)
    double* gE;
    double* gV;                         // row parts per band: [R][nb][row_stride]
    double* gR;
    int64_t R;
    int nb;                             // band slots per realisation in gV / gR
    int max_n;                          // largest chain of the batch (the grid's bands)
    int row_stride;
    int levels;                         // K
    int dtype;
    int periodic;
    int layout;                         // 0: one row, 1: full grid, 2: triangle (bosons)
    int contract;                       // 1: contract every level's input with v
};

// Output columns of a band of a K-level pass.
inline int pipe_band_width(int K) { return 64 - 2 * K; }
inline int pipe_max_levels(int dtype, bool contract) {
    if (contract) return dtype == 1 ? kPipeMaxHornerC128 : kPipeMaxHornerC64;
    return dtype == 1 ? kPipeMaxLevelsC128 : kPipeMaxLevelsC64;
}

hipError_t launch_adj_pipe(const AdjPipeArgs& a, hipStream_t stream);

}  // namespace ctqw
