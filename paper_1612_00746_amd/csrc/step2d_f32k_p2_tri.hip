// Compiled pipeline depths: float state, 2 column(s) per lane, Kahan accumulation, boson triangle layout.
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f32k_p2_tri(int levels) {
    switch (levels) {
        CTQW_STEP_CASE(float, 1, 2, true, true)
        CTQW_STEP_CASE(float, 2, 2, true, true)
        CTQW_STEP_CASE(float, 3, 2, true, true)
        CTQW_STEP_CASE(float, 4, 2, true, true)
        CTQW_STEP_CASE(float, 5, 2, true, true)
        CTQW_STEP_CASE(float, 6, 2, true, true)
        CTQW_STEP_CASE(float, 7, 2, true, true)
        CTQW_STEP_CASE(float, 8, 2, true, true)
        CTQW_STEP_CASE(float, 9, 2, true, true)
        default: return nullptr;
    }
}
}  // namespace ctqw
