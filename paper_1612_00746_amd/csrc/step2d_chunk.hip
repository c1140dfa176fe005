// Chunked steps: passes of chunk_depth(dtype) terms for Taylor orders above
// the fused pipeline's compiled depth (one column per lane).
#include "step2d_impl.hpp"

namespace ctqw {

namespace {

StepKernelFn select_chunk(const StepConfig& c) {
    using namespace step2d_detail;
    constexpr int D = chunk_depth(0), D64 = chunk_depth(1);
    if (c.cols_per_lane != 1) return nullptr;
    if (c.dtype == 1) return c.triangle ? &step2d_kernel<double, D64, 1, false, true, true>
                                        : &step2d_kernel<double, D64, 1, false, false, true>;
    if (c.kahan) return c.triangle ? &step2d_kernel<float, D, 1, true, true, true>
                                   : &step2d_kernel<float, D, 1, true, false, true>;
    return c.triangle ? &step2d_kernel<float, D, 1, false, true, true> : &step2d_kernel<float, D, 1, false, false, true>;
}

}  // namespace

hipError_t launch_chunk_pass(const StepConfig& cfg, const StepArgs& args, hipStream_t stream) {
    StepKernelFn fn = select_chunk(cfg);
    if (!fn) return hipErrorInvalidValue;
    const int wpb = cfg.waves_per_block;
    const int blocks = cfg.persistent ? cfg.grid_blocks : (args.n_items + wpb - 1) / wpb;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * wpb), 0, stream, args);
    return hipGetLastError();
}

hipError_t chunk_max_block(const StepConfig& cfg, int* threads) {
    StepKernelFn fn = select_chunk(cfg);
    if (!fn) return hipErrorInvalidValue;
    hipFuncAttributes attr{};
    hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(fn));
    if (e == hipSuccess) *threads = attr.maxThreadsPerBlock;
    return e;
}

hipError_t chunk_occupancy(const StepConfig& cfg, int* blocks_per_cu) {
    StepKernelFn fn = select_chunk(cfg);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(fn),
                                                        cfg.waves_per_block * 64, 0);
}

}  // namespace ctqw
