// Time-dependent (switching) hopping noise (see telegraph.hip).
#pragma once
#include "ctqw_internal.hpp"

namespace ctqw {

struct TeleArgs {
    const RealDev* reals;
    const double* Jbase;         // [param_total] baseline hoppings (unscaled)
    float* sign;                 // [param_total] current sign of xi per bond
    int32_t* step;               // steps taken since the switching process started
    double* Jd;                  // [param_total] dt * J, updated
    float* Jf;
    double dt, amp, p_flip;
    uint32_t key0, key1;
    int64_t R;
};
hipError_t launch_telegraph(const TeleArgs& a, int max_bonds, hipStream_t s);

}  // namespace ctqw
