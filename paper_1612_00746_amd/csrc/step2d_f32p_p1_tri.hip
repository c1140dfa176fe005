// Compiled pipeline depths: float state, 1 column(s) per lane, plain accumulation, boson triangle layout.
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f32p_p1_tri(int levels) {
    switch (levels) {
        CTQW_STEP_CASE(float, 1, 1, false, true)
        CTQW_STEP_CASE(float, 2, 1, false, true)
        CTQW_STEP_CASE(float, 3, 1, false, true)
        CTQW_STEP_CASE(float, 4, 1, false, true)
        CTQW_STEP_CASE(float, 5, 1, false, true)
        CTQW_STEP_CASE(float, 6, 1, false, true)
        CTQW_STEP_CASE(float, 7, 1, false, true)
        CTQW_STEP_CASE(float, 8, 1, false, true)
        CTQW_STEP_CASE(float, 9, 1, false, true)
        CTQW_STEP_CASE(float, 10, 1, false, true)
        CTQW_STEP_CASE(float, 11, 1, false, true)
        CTQW_STEP_CASE(float, 12, 1, false, true)
        default: return nullptr;
    }
}
}  // namespace ctqw
