// Compiled pipeline depths: float state, 2 columns per lane, Kahan accumulation, full grid layout,
// one 16-byte access per lane (items whose column pairs are adjacent in memory).
#include "step2d_impl.hpp"

namespace ctqw {
StepKernelFn step_table_f32k_p2_vec(int levels) {
    switch (levels) {
        CTQW_STEP_CASE_VEC(float, 1, true)
        CTQW_STEP_CASE_VEC(float, 2, true)
        CTQW_STEP_CASE_VEC(float, 3, true)
        CTQW_STEP_CASE_VEC(float, 4, true)
        CTQW_STEP_CASE_VEC(float, 5, true)
        CTQW_STEP_CASE_VEC(float, 6, true)
        CTQW_STEP_CASE_VEC(float, 7, true)
        CTQW_STEP_CASE_VEC(float, 8, true)
        CTQW_STEP_CASE_VEC(float, 9, true)
        default: return nullptr;
    }
}
}  // namespace ctqw
