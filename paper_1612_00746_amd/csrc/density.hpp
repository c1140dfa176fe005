// Ensemble-averaged density matrix (see density.hip).
#pragma once
#include "ctqw_internal.hpp"

namespace ctqw {

// Density matrix of one group: gather of the members' states.
struct DensityArgs {
    const void* psi;
    const RealDev* reals;
    const double* scale;
    const int32_t* members;      // [R_g] realisation indices (device)
    void* A;                     // [R_g][D] gathered, scaled states
    int64_t D;
    int64_t R_g;
    int triangle;                // bosons: sqrt(2) weight off the diagonal
};
hipError_t launch_density_gather(const DensityArgs& a, int dtype, hipStream_t s);
hipError_t launch_density_mirror(void* rho, int64_t D, int64_t ld, int dtype, hipStream_t s);
int density_herk(void** handle, hipStream_t s, int dtype, int64_t D, int64_t R_g, const void* A, void* rho,
                 int64_t ld);
void density_release(void* handle);


}  // namespace ctqw
