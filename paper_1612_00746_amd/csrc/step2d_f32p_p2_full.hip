// Compiled pipeline depths: float state, 2 column(s) per lane, plain accumulation, full grid layout.
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f32p_p2_full(int levels) {
    switch (levels) {
        CTQW_STEP_CASE(float, 1, 2, false, false)
        CTQW_STEP_CASE(float, 2, 2, false, false)
        CTQW_STEP_CASE(float, 3, 2, false, false)
        CTQW_STEP_CASE(float, 4, 2, false, false)
        CTQW_STEP_CASE(float, 5, 2, false, false)
        CTQW_STEP_CASE(float, 6, 2, false, false)
        CTQW_STEP_CASE(float, 7, 2, false, false)
        CTQW_STEP_CASE(float, 8, 2, false, false)
        CTQW_STEP_CASE(float, 9, 2, false, false)
        default: return nullptr;
    }
}
}  // namespace ctqw
