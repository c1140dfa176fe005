// Compiled pipeline depths for launches holding two orders (n and n - 1): float state,
// 2 columns per lane, full grid, one 16-byte access per lane, plain accumulation.
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f32p_p2_vec_two(int levels) {
    switch (levels) {
        CTQW_STEP_CASE_TWO(float, 2, 2, false, true)
        CTQW_STEP_CASE_TWO(float, 3, 2, false, true)
        CTQW_STEP_CASE_TWO(float, 4, 2, false, true)
        CTQW_STEP_CASE_TWO(float, 5, 2, false, true)
        CTQW_STEP_CASE_TWO(float, 6, 2, false, true)
        CTQW_STEP_CASE_TWO(float, 7, 2, false, true)
        CTQW_STEP_CASE_TWO(float, 8, 2, false, true)
        CTQW_STEP_CASE_TWO(float, 9, 2, false, true)
        default: return nullptr;
    }
}
}  // namespace ctqw
