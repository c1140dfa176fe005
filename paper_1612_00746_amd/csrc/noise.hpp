// Host-side noise draws (see noise.hip).
#pragma once
#include <stdint.h>

#include "../../include/ctqw.h"

namespace ctqw {

// Kinds of parameters in the generator's counter.
enum : int { NOISE_BOND = 0, NOISE_SITE = 1, NOISE_INTERACTION = 2 };

// One Philox4x32-10 block.
void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
// 53-bit uniform in [0, 1) from two words.
double unit_double(uint32_t hi, uint32_t lo);
// The stochastic part of parameter `index` of kind `kind` in realisation r.
double noise_draw(const ctqw_noise& n, uint64_t seed, int64_t r, int kind, int64_t index);

}  // namespace ctqw
