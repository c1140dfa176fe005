// Ensemble-averaged density matrix (see density.hip).
#pragma once
#include "ctqw_internal.hpp"

namespace ctqw {

// Density matrix of one group: gather of the members' states into split
// planes [re / im][Rp][Dp] (realisation-major, zero padding up to Dp rows
// and Rp realisations).
struct DensityArgs {
    const void* psi;
    const RealDev* reals;
    const double* scale;
    const int32_t* members;      // [R_g] realisation indices (device)
    void* A;                     // [2][Rp][Dp] gathered, scaled states
    int64_t D;
    int64_t R_g;
    int64_t Dp;                  // padded rows (multiple of the tile)
    int64_t Rp;                  // padded realisations (multiple of the stage)
    int triangle;                // bosons, fermions: sqrt(2) weight off the diagonal
};
hipError_t launch_density_gather(const DensityArgs& a, int dtype, hipStream_t s);
hipError_t launch_density_mirror(void* rho, int64_t D, int64_t ld, int dtype, hipStream_t s);

// rho (lower triangle, column-major, ld) = A A^H / R from the gathered planes.
struct HerkArgs {
    const void* G;               // [2][Rp][Dp] real / imaginary planes
    void* rho;
    int64_t D, Dp, ld;
    int32_t Rp;
    int64_t n_tiles;             // T (T + 1) / 2 with T = Dp / tile
    double inv_R;
};
int herk_tile(int dtype);        // rows of a tile (128 complex64, 64 complex128)
int herk_stage(int dtype);       // realisations per LDS stage
hipError_t launch_herk(const HerkArgs& a, int dtype, hipStream_t s);


}  // namespace ctqw
