// Time-dependent hopping noise (Eq. 1 with switching stochastic terms):
// every bond of every realisation carries xi(t) = +-a, flipping sign at
// the events of a Poisson process of rate g.  Discretised per step: at the
// start of step s each bond flips with probability 1 - exp(-g dt) and the
// resulting J = Jbar + xi holds during the step.
//
// Draws: Philox4x32-10 (Salmon et al., SC 2011) with counter (bond index,
// 4 (s + 1), r mod 2^32, r div 2^32) and key (seed_lo XOR 0x54454C45,
// seed_hi); u = 53-bit fraction of (w0, w1).  s = -1 gives the initial sign
// (+a if u < 1/2), drawn on the host at upload.
#include "telegraph.hpp"

namespace ctqw {
namespace {

__device__ __forceinline__ void philox_device(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t& w0, uint32_t& w1) {
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    w0 = c0;
    w1 = c1;
}

// One bond of realisation r: the flip test of the current step, the new sign
// and the bond's dt-scaled table entries.
__device__ void flip_bond(const TeleArgs& a, const RealDev& rd, int64_t r, int i) {
    const int64_t k = rd.param_off + i;
    const int32_t s = *a.step;
    uint32_t w0, w1;
    philox_device((uint32_t)i, 4u * (uint32_t)(s + 1), (uint32_t)((uint64_t)r & 0xffffffffu),
                  (uint32_t)((uint64_t)r >> 32), a.key0, a.key1, w0, w1);
    const double u = ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6)) * (1.0 / 9007199254740992.0);
    float sg = a.sign[k];
    if (u < a.p_flip) sg = -sg;
    a.sign[k] = sg;
    const double Jdt = a.dt * (a.Jbase[k] + a.amp * (double)sg);
    a.Jd[k] = Jdt;
    a.Jf[k] = (float)Jdt;
}

// thread per bond; realisations strided over the grid's second dimension
__global__ void telegraph_kernel(TeleArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t r = blockIdx.y; r < a.R; r += gridDim.y) {
        const RealDev rd = a.reals[r];
        const int nb = (rd.flags & RF_PERIODIC) ? rd.N : rd.N - 1;
        if (i < nb) flip_bond(a, rd, r, i);
    }
}

__global__ void step_count_kernel(int32_t* step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

}  // namespace

hipError_t launch_telegraph(const TeleArgs& a, int max_bonds, hipStream_t s) {
    if (a.R <= 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((max_bonds + 255) / 256), (unsigned)(a.R < 65535 ? a.R : 65535));
    hipLaunchKernelGGL(telegraph_kernel, grid, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(step_count_kernel, dim3(1), dim3(64), 0, s, a.step);
    return hipGetLastError();
}

}  // namespace ctqw
