// Selection of the compiled step kernel for a launch configuration.
#include "step2d_impl.hpp"

namespace ctqw {

#define CTQW_DECLARE_TABLE(tag) StepKernelFn step_table_##tag(int levels);
CTQW_DECLARE_TABLE(f32k_p1_full) CTQW_DECLARE_TABLE(f32k_p1_tri)
CTQW_DECLARE_TABLE(f32k_p2_full) CTQW_DECLARE_TABLE(f32k_p2_tri)
CTQW_DECLARE_TABLE(f32p_p1_full) CTQW_DECLARE_TABLE(f32p_p1_tri)
CTQW_DECLARE_TABLE(f32p_p2_full) CTQW_DECLARE_TABLE(f32p_p2_tri)
CTQW_DECLARE_TABLE(f64_p1_full) CTQW_DECLARE_TABLE(f64_p1_tri)
CTQW_DECLARE_TABLE(f64_p2_full) CTQW_DECLARE_TABLE(f64_p2_tri)
CTQW_DECLARE_TABLE(f32k_p2_vec) CTQW_DECLARE_TABLE(f32p_p2_vec)
CTQW_DECLARE_TABLE(f32k_p2_full_two) CTQW_DECLARE_TABLE(f32k_p2_vec_two)
CTQW_DECLARE_TABLE(f32p_p2_full_two) CTQW_DECLARE_TABLE(f32p_p2_vec_two)
#undef CTQW_DECLARE_TABLE

namespace {

// Deepest compiled pipeline per (dtype, columns per lane); every depth from
// 1 up to it is compiled (see the step2d_*.hip tables).  Deeper pipelines
// spill to scratch memory; their orders run as chunked passes.
int max_levels(int dtype, int cols_per_lane) {
    if (dtype == 1) return cols_per_lane == 1 ? 12 : 7;
    return cols_per_lane == 1 ? 12 : 9;
}

StepKernelFn select_kernel(const StepConfig& c) {
    const bool t = c.triangle != 0;
    if (c.cols_per_lane != 1 && c.cols_per_lane != 2) return nullptr;
    const bool p1 = c.cols_per_lane == 1;
    if (c.dtype == 1)
        return p1 ? (t ? step_table_f64_p1_tri(c.levels) : step_table_f64_p1_full(c.levels))
                  : (t ? step_table_f64_p2_tri(c.levels) : step_table_f64_p2_full(c.levels));
    if (c.two) {
        // two orders per launch: complex64 full grid, two columns per lane
        if (t || p1) return nullptr;
        if (c.kahan) return c.vec ? step_table_f32k_p2_vec_two(c.levels) : step_table_f32k_p2_full_two(c.levels);
        return c.vec ? step_table_f32p_p2_vec_two(c.levels) : step_table_f32p_p2_full_two(c.levels);
    }
    if (c.vec) {
        if (t || p1) return nullptr;
        return c.kahan ? step_table_f32k_p2_vec(c.levels) : step_table_f32p_p2_vec(c.levels);
    }
    if (c.kahan)
        return p1 ? (t ? step_table_f32k_p1_tri(c.levels) : step_table_f32k_p1_full(c.levels))
                  : (t ? step_table_f32k_p2_tri(c.levels) : step_table_f32k_p2_full(c.levels));
    return p1 ? (t ? step_table_f32p_p1_tri(c.levels) : step_table_f32p_p1_full(c.levels))
              : (t ? step_table_f32p_p2_tri(c.levels) : step_table_f32p_p2_full(c.levels));
}

}  // namespace

int step_levels_bucket(int dtype, int cols_per_lane, int order) {
    if (order < 1 || (cols_per_lane != 1 && cols_per_lane != 2)) return -1;
    return order <= max_levels(dtype, cols_per_lane) ? order : -1;
}

hipError_t step_occupancy(const StepConfig& cfg, int* blocks_per_cu) {
    StepKernelFn fn = select_kernel(cfg);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(fn),
                                                        cfg.waves_per_block * 64, 0);
}

hipError_t step_max_block(const StepConfig& cfg, int* threads) {
    StepKernelFn fn = select_kernel(cfg);
    if (!fn) return hipErrorInvalidValue;
    hipFuncAttributes attr{};
    hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(fn));
    if (e == hipSuccess) *threads = attr.maxThreadsPerBlock;
    return e;
}

hipError_t launch_step(const StepConfig& cfg, const StepArgs& args, hipStream_t stream) {
    StepKernelFn fn = select_kernel(cfg);
    if (!fn) return hipErrorInvalidValue;
    const int wpb = cfg.waves_per_block;
    const int blocks = cfg.persistent ? cfg.grid_blocks : (args.n_items + wpb - 1) / wpb;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * wpb), 0, stream, args);
    return hipGetLastError();
}

}  // namespace ctqw
