// Compiled pipeline depths: double state, 2 column(s) per lane, plain accumulation, boson triangle layout.
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f64_p2_tri(int levels) {
    switch (levels) {
        CTQW_STEP_CASE(double, 1, 2, false, true)
        CTQW_STEP_CASE(double, 2, 2, false, true)
        CTQW_STEP_CASE(double, 3, 2, false, true)
        CTQW_STEP_CASE(double, 4, 2, false, true)
        CTQW_STEP_CASE(double, 5, 2, false, true)
        CTQW_STEP_CASE(double, 6, 2, false, true)
        CTQW_STEP_CASE(double, 7, 2, false, true)
        default: return nullptr;
    }
}
}  // namespace ctqw
