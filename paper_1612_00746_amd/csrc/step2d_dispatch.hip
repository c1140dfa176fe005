// Selection of the compiled step kernel for a launch configuration.
#include "step2d_impl.hpp"

namespace ctqw {

StepKernelFn step_table_f32k_p1(int levels);
StepKernelFn step_table_f32k_p2(int levels);
StepKernelFn step_table_f32p_p1(int levels);
StepKernelFn step_table_f32p_p2(int levels);
StepKernelFn step_table_f64_p1(int levels);
StepKernelFn step_table_f64_p2(int levels);

namespace {

// Compiled depths, ascending; must match the step2d_*.hip tables.
constexpr int kLevels32[] = {3, 4, 5, 6, 7, 8, 10, 12};
constexpr int kLevels64p1[] = {3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 16};
constexpr int kLevels64p2[] = {3, 4, 5, 6, 7, 8};

StepKernelFn select_kernel(const StepConfig& c) {
    if (c.dtype == 1) {
        return c.cols_per_lane == 1 ? step_table_f64_p1(c.levels)
                                    : (c.cols_per_lane == 2 ? step_table_f64_p2(c.levels) : nullptr);
    }
    if (c.kahan) {
        return c.cols_per_lane == 1 ? step_table_f32k_p1(c.levels)
                                    : (c.cols_per_lane == 2 ? step_table_f32k_p2(c.levels) : nullptr);
    }
    return c.cols_per_lane == 1 ? step_table_f32p_p1(c.levels)
                                : (c.cols_per_lane == 2 ? step_table_f32p_p2(c.levels) : nullptr);
}

}  // namespace

int step_levels_bucket(int dtype, int cols_per_lane, int order) {
    if (order < 1) return -1;
    if (dtype == 1) {
        if (cols_per_lane == 2) {
            for (int v : kLevels64p2) if (v >= order) return v;
            return -1;
        }
        for (int v : kLevels64p1) if (v >= order) return v;
        return -1;
    }
    for (int v : kLevels32) if (v >= order) return v;
    return -1;
}

hipError_t step_occupancy(const StepConfig& cfg, int* blocks_per_cu) {
    StepKernelFn fn = select_kernel(cfg);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(fn),
                                                        cfg.waves_per_block * 64, 0);
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
