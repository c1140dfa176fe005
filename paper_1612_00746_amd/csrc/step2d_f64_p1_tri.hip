// Compiled pipeline depths: double state, 1 column(s) per lane, plain accumulation, boson triangle layout.
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f64_p1_tri(int levels) {
    switch (levels) {
        CTQW_STEP_CASE(double, 1, 1, false, true)
        CTQW_STEP_CASE(double, 2, 1, false, true)
        CTQW_STEP_CASE(double, 3, 1, false, true)
        CTQW_STEP_CASE(double, 4, 1, false, true)
        CTQW_STEP_CASE(double, 5, 1, false, true)
        CTQW_STEP_CASE(double, 6, 1, false, true)
        CTQW_STEP_CASE(double, 7, 1, false, true)
        CTQW_STEP_CASE(double, 8, 1, false, true)
        CTQW_STEP_CASE(double, 9, 1, false, true)
        CTQW_STEP_CASE(double, 10, 1, false, true)
        CTQW_STEP_CASE(double, 11, 1, false, true)
        CTQW_STEP_CASE(double, 12, 1, false, true)
        default: return nullptr;
    }
}
}  // namespace ctqw
