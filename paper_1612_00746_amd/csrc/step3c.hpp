// Product form of the three-particle step.
//
// The step's Taylor polynomial p_n(z) = sum_{k<=n} z^k / k! (z = -i dt H,
// Eqs. 6-7) has p_n(0) = 1 and n roots z_k, so p_n(z) = prod_k (1 - z / z_k)
// (the same polynomial: the map differs from the chained sum by rounding
// only).  Split into one group of at most K factors per pass, each pass maps
// its input X to q(z) X = X + sum_j e_j z^j X = X + sum_j c_j Y_j with
// Y_j = (dt H)^j X and c_j = e_j (-i)^j, e_j the elementary symmetric
// polynomials of -1/z_k over the pass's roots.  A pass then reads one state
// and writes one (16 B per amplitude in complex64), where the chained sum
// also carries the partial sum and the seed of the next pass between passes.
//
// The last term's norm, which the truncation test compares with the
// tolerance, is not formed on the way: with the first pass's K levels, the
// step bounds it by ||(dt H)^n psi|| <= (dt G)^(n-K) ||(dt H)^K psi|| (G the
// Gershgorin bound on ||H||_2 that chose the order), an upper bound.
#pragma once

#include "ctqw_internal.hpp"

namespace ctqw {

struct Step3cProd {
    double cre[4];     // Re c_j, j = 1 .. K
    double cim[4];     // Im c_j
    int32_t order;     // n
    int32_t k_first;   // levels of the step's first pass
};

// One pass of the product form (the Step3cArgs seed and partial-sum fields
// are unused; first / last as for the chained passes).
hipError_t launch_step3c_prod(const Step3cArgs& a, const Step3cProd& pp, int dtype, int K, hipStream_t stream);

}  // namespace ctqw
