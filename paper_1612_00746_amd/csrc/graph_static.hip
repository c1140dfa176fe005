// ctqw_graph_evolve_static: the general-graph propagation of
// ctqw_graph_evolve (Sec. 2, Eqs. 5-7) for callers that cannot allocate
// device memory.  Its scratch -- the two term buffers and the partial sum of
// the one-term-per-pass series -- is a file-scope device array of fixed
// size instead of a caller-provided workspace; every other argument and the
// kernels are those of ctqw_graph_evolve.
//
// Each device holds its own copy of the array from the time the library's
// code object is loaded on it until the process ends.  The array's address
// on a device is looked up once per device (hipGetSymbolAddress with that
// device current) and kept; the host-side name of the array is never used
// as a device address.  Every call on one device shares that device's
// array: calls that overlap on one device (different streams, or other
// host threads) race.  Nothing in the array has to start at zero: every
// pass writes the buffers it later reads.
#include <cstdio>
#include <mutex>

#include "../../include/ctqw.h"
#include "ctqw_internal.hpp"

namespace {

constexpr int64_t kScratchBytes = CTQW_GRAPH_STATIC_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on device dev (looked up once).
hipError_t scratch_on(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" ctqw_status ctqw_graph_evolve_static(int32_t n_nodes, int32_t width, const int32_t* nbr, const void* hop,
                                                const void* onsite, int32_t R, int32_t dtype, double dt, int32_t order,
                                                int64_t n_steps, void* psi, double* norms, void* hip_stream) {
    int64_t need = 0;
    const ctqw_status st = ctqw_graph_workspace(n_nodes, R, dtype, &need);
    if (st != CTQW_OK) return st;
    if (need > kScratchBytes) {
        char msg[256];
        snprintf(msg, sizeof msg,
                 "ctqw_graph_evolve_static: %lld scratch bytes needed, the static buffer holds %lld "
                 "(use ctqw_graph_evolve with a workspace)",
                 (long long)need, (long long)kScratchBytes);
        return (ctqw_status)ctqw::report_error(CTQW_ERR_UNSUPPORTED, msg);
    }
    if (width < 0 || !onsite || !psi || (width > 0 && (!nbr || !hop)))
        return (ctqw_status)ctqw::report_error(CTQW_ERR_INVALID_ARG, "ctqw_graph_evolve_static: NULL argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int dev = 0;
    hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
    void* ws = nullptr;
    if (e == hipSuccess) e = scratch_on(dev, &ws);
    if (e != hipSuccess) {
        char msg[256];
        snprintf(msg, sizeof msg, "ctqw_graph_evolve_static: scratch lookup failed: %s", hipGetErrorString(e));
        return (ctqw_status)ctqw::report_error(CTQW_ERR_DEVICE, msg);
    }
    return ctqw_graph_evolve(n_nodes, width, nbr, hop, onsite, R, dtype, dt, order, n_steps, psi, ws, kScratchBytes,
                             norms, hip_stream);
}
