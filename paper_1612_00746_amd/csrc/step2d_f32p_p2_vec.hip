// Compiled pipeline depths: float state, 2 columns per lane, plain accumulation, full grid layout,
// one 16-byte access per lane (items whose column pairs are adjacent in memory).
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f32p_p2_vec(int levels) {
    switch (levels) {
        CTQW_STEP_CASE_VEC(float, 1, false)
        CTQW_STEP_CASE_VEC(float, 2, false)
        CTQW_STEP_CASE_VEC(float, 3, false)
        CTQW_STEP_CASE_VEC(float, 4, false)
        CTQW_STEP_CASE_VEC(float, 5, false)
        CTQW_STEP_CASE_VEC(float, 6, false)
        CTQW_STEP_CASE_VEC(float, 7, false)
        CTQW_STEP_CASE_VEC(float, 8, false)
        CTQW_STEP_CASE_VEC(float, 9, false)
        default: return nullptr;
    }
}
}  // namespace ctqw
