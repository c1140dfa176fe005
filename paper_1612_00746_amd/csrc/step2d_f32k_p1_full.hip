// Compiled pipeline depths: float state, 1 column(s) per lane, Kahan accumulation, full grid layout.
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f32k_p1_full(int levels) {
    switch (levels) {
        CTQW_STEP_CASE(float, 1, 1, true, false)
        CTQW_STEP_CASE(float, 2, 1, true, false)
        CTQW_STEP_CASE(float, 3, 1, true, false)
        CTQW_STEP_CASE(float, 4, 1, true, false)
        CTQW_STEP_CASE(float, 5, 1, true, false)
        CTQW_STEP_CASE(float, 6, 1, true, false)
        CTQW_STEP_CASE(float, 7, 1, true, false)
        CTQW_STEP_CASE(float, 8, 1, true, false)
        CTQW_STEP_CASE(float, 9, 1, true, false)
        CTQW_STEP_CASE(float, 10, 1, true, false)
        CTQW_STEP_CASE(float, 11, 1, true, false)
        CTQW_STEP_CASE(float, 12, 1, true, false)
        default: return nullptr;
    }
}
}  // namespace ctqw
