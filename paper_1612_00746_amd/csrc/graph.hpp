// One particle on a general graph (see graph.hip).
#pragma once
#include "ctqw_internal.hpp"

namespace ctqw {

// One Taylor term of every realisation: t = (-i c) H src, acc_out = acc_in + t.
// Pointers are untyped: complex64 states with FP32 tables, or complex128
// states with FP64 tables (dtype 0 / 1).
struct GraphTermArgs {
    const int32_t* nbr;      // [width][n] neighbour of node i in slot k; outside [0, n): empty slot
    const void* hop;         // [R][width][n] coupling of that slot
    const void* onsite;      // [R][n] diagonal
    const void* src;         // [R][n] the previous term (or the state)
    void* t_out;             // [R][n] this term, or NULL when no later term needs it
    const void* acc_in;      // [R][n] partial sum before this term
    void* acc_out;           // [R][n] partial sum after it
    double c;                // dt / j for term j
    int32_t n;
    int32_t width;
    int32_t R;
};
hipError_t launch_graph_term(const GraphTermArgs& a, int dtype, hipStream_t s);
// out[r] = sum_i |psi[r][i]|^2 in FP64, one block per realisation, fixed summation order.
hipError_t launch_graph_norms(const void* psi, int32_t n, int32_t R, double* out, int dtype, hipStream_t s);

}  // namespace ctqw
