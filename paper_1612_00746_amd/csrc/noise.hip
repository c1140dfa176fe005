// Host-side draws of the static noise (Eq. 1: every parameter is a
// deterministic baseline plus a stochastic part, here fixed in time).
//
// Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  One block of
// four 32-bit words per parameter, counter = (index, kind, r_lo, r_hi) with
// kind 0 for bond hoppings, 1 for on-site energies, 2 for the interaction,
// key = (seed_lo, seed_hi).  Any parameter of any realisation is therefore
// drawn on its own, independently of the batch it sits in.
//
// From a block (w0, w1, w2, w3):
//   u = (2^26 * (w0 >> 5) + (w1 >> 6)) * 2^-53      in [0, 1)
//   v = (2^26 * (w2 >> 5) + (w3 >> 6)) * 2^-53
//   uniform U[a, b] : a + (b - a) * u
//   normal N(a, b^2): a + b * sqrt(-2 log(1 - u)) * cos(2 pi v)   (Box-Muller)
// evaluated without contraction, so a plain double evaluation elsewhere
// gives the same bits.
#include "../../include/ctqw.h"
#include "noise.hpp"

#include <cmath>

namespace ctqw {

void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;   // round multipliers
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u; // key schedule increments
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        const uint64_t p0 = (uint64_t)kMul0 * c0;
        const uint64_t p1 = (uint64_t)kMul1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

double unit_double(uint32_t hi, uint32_t lo) {
    const double k = 67108864.0 * (double)(hi >> 5) + (double)(lo >> 6);   // exact: < 2^53
    return k * (1.0 / 9007199254740992.0);
}

#pragma clang fp contract(off)
double noise_draw(const ctqw_noise& n, uint64_t seed, int64_t r, int kind, int64_t index) {
    if (n.dist == CTQW_DIST_NONE) return 0.0;
    const uint32_t ctr[4] = {(uint32_t)index, (uint32_t)kind, (uint32_t)((uint64_t)r & 0xffffffffu),
                             (uint32_t)((uint64_t)r >> 32)};
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    const double u = unit_double(w[0], w[1]);
    if (n.dist == CTQW_DIST_UNIFORM) {
        const double span = n.b - n.a;
        const double t = span * u;
        return n.a + t;
    }
    const double v = unit_double(w[2], w[3]);
    const double radius = std::sqrt(-2.0 * std::log(1.0 - u));
    const double angle = 6.283185307179586 * v;
    const double z = radius * std::cos(angle);
    const double t = n.b * z;
    return n.a + t;
}

}  // namespace ctqw
