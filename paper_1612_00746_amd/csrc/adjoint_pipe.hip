// Launcher of the K-level adjoint passes (kernel in adjoint_pipe_impl.hpp).
#include "adjoint_pipe_impl.hpp"

#include <climits>
#include <utility>

namespace ctqw {
namespace {

using PipeFn = void (*)(AdjPipeArgs);

template <typename T, int LAY, bool PER, bool CON, int... Ks>
PipeFn pick_levels(int K, std::integer_sequence<int, Ks...>) {
    PipeFn fn = nullptr;
    ((fn = (K == Ks + 1) ? &adj_pipe::pipe_kernel<T, Ks + 1, LAY, PER, CON> : fn), ...);
    return fn;
}

template <typename T, int KMAX, int HMAX>
PipeFn pick(const AdjPipeArgs& a) {
    const auto ks = std::make_integer_sequence<int, KMAX>{};
    const auto hs = std::make_integer_sequence<int, HMAX>{};
    const bool con = a.contract != 0;
    const int K = a.levels;
    switch (a.layout * 2 + (a.periodic ? 1 : 0)) {
    case 0: return con ? pick_levels<T, 0, false, true>(K, hs) : pick_levels<T, 0, false, false>(K, ks);
    case 1: return con ? pick_levels<T, 0, true, true>(K, hs) : pick_levels<T, 0, true, false>(K, ks);
    case 2: return con ? pick_levels<T, 1, false, true>(K, hs) : pick_levels<T, 1, false, false>(K, ks);
    case 3: return con ? pick_levels<T, 1, true, true>(K, hs) : pick_levels<T, 1, true, false>(K, ks);
    case 4: return con ? pick_levels<T, 2, false, true>(K, hs) : pick_levels<T, 2, false, false>(K, ks);
    default: return nullptr;   // no triangle on a ring
    }
}

}  // namespace

hipError_t launch_adj_pipe(const AdjPipeArgs& a, hipStream_t s) {
    if (a.R < 1 || a.R > 65535 || a.nb < 1 || a.nb > 65535) return hipErrorInvalidValue;
    if (a.levels < 1 || a.levels > pipe_max_levels(a.dtype, a.contract != 0) || a.layout < 0 || a.layout > 2)
        return hipErrorInvalidValue;
    if (a.contract && (!a.gJ || !a.gE || !a.gV || !a.gR)) return hipErrorInvalidValue;
    // the kernels store every level of a forward pass and only the last of a
    // contracting (Horner) pass
    for (int l = 0; l < a.levels; ++l)
        if ((a.y[l] != nullptr) != (!a.contract || l == a.levels - 1)) return hipErrorInvalidValue;
    // one buffer resource spans a realisation's amplitudes
    const int64_t amps = a.layout == 0 ? (int64_t)a.max_n : (int64_t)a.max_n * a.max_n;
    if (amps * (a.dtype == 1 ? 16 : 8) > INT32_MAX) return hipErrorInvalidValue;
    const PipeFn fn = a.dtype == 1 ? pick<double, kPipeMaxLevelsC128, kPipeMaxHornerC128>(a)
                                   : pick<float, kPipeMaxLevelsC64, kPipeMaxHornerC64>(a);
    if (!fn) return hipErrorInvalidValue;
    // bands of the largest chain; a contracting pass has a row-part slot for each
    const int W = pipe_band_width(a.levels);
    const int bands = (a.max_n + W - 1) / W;
    if (a.max_n < 1 || (a.contract && bands > a.nb)) return hipErrorInvalidValue;
    const dim3 g((unsigned)bands, (unsigned)a.R);
    hipLaunchKernelGGL(fn, g, dim3(64 * kSweepSegs), 0, s, a);
    return hipGetLastError();
}

}  // namespace ctqw
