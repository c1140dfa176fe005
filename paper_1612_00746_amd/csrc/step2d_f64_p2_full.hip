// Compiled pipeline depths: double state, 2 column(s) per lane, plain accumulation, full grid layout.
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f64_p2_full(int levels) {
    switch (levels) {
        CTQW_STEP_CASE(double, 1, 2, false, false)
        CTQW_STEP_CASE(double, 2, 2, false, false)
        CTQW_STEP_CASE(double, 3, 2, false, false)
        CTQW_STEP_CASE(double, 4, 2, false, false)
        CTQW_STEP_CASE(double, 5, 2, false, false)
        CTQW_STEP_CASE(double, 6, 2, false, false)
        CTQW_STEP_CASE(double, 7, 2, false, false)
        default: return nullptr;
    }
}
}  // namespace ctqw
