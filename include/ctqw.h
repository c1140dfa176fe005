/*
 * ctqw.h -- C ABI of libctqw, an MI355X (gfx950) implementation of the
 * truncated-Taylor propagation of many noisy realisations of a
 * many-particle tight-binding walk, after Piccinini et al., "GPU-accelerated
 * algorithms for many-particle continuous-time quantum walks"
 * (arXiv:1612.00746).
 *
 * The problem statement follows Sec. 2 of the paper: m particles on a
 * one-dimensional lattice of N nodes (q = 1, nearest-neighbour hopping),
 * Hamiltonian entries made of a deterministic and a stochastic part on the
 * diagonal and between neighbours (Eq. 1), R independent realisations whose
 * density matrices are averaged (Eq. 2), and the evolution operator
 * exp(-i H dt) expanded in a Taylor series (Eqs. 5-7, Alg. 3).  hbar = 1.
 *
 * Conventions shared by every entry point
 *  - Every function returns ctqw_status; nothing else crosses the ABI.
 *    Output arguments come last.
 *  - Host arrays passed in are copied before the call returns.
 *  - Device memory (the two state buffers and the workspace) is owned by
 *    the caller; the library never allocates or frees device memory.
 *    Sizes come from ctqw_sizes().
 *  - Work is enqueued on the stream given to ctqw_bind().  Calls that return
 *    host data (ctqw_propagate, ctqw_observe, ctqw_get_state, ctqw_stats,
 *    ctqw_realization_norms) synchronise that stream; device faults and the
 *    norm / truncation alarms are reported by those calls.
 *  - A plan is not thread-safe.  Distinct plans are independent.
 *  - On CTQW_ERR_INVALID_ARG the plan is left unchanged; ctqw_last_error()
 *    returns a description of the last failure on a plan.
 */
#ifndef CTQW_H
#define CTQW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CTQW_OK = 0,
    CTQW_ERR_INVALID_ARG = 1,   /* bad pointer, size, enum or non-finite value */
    CTQW_ERR_UNSUPPORTED = 2,   /* valid request this build does not implement */
    CTQW_ERR_OUT_OF_MEMORY = 3, /* host allocation failed or sizes overflow */
    CTQW_ERR_DEVICE = 4,        /* a HIP runtime call failed */
    CTQW_ERR_NOT_CONVERGED = 5, /* Taylor order above the cap, or the FP64
                                   a-posteriori truncation test failed */
    CTQW_ERR_NUMERICAL = 6,     /* non-finite state or norm outside the alarm */
    CTQW_ERR_STATE = 7          /* call out of order (e.g. propagate before bind) */
} ctqw_status;

/* Particle statistics (Sec. 1 of the paper: walks depend on statistics). */
typedef enum { CTQW_DISTINGUISHABLE = 0, CTQW_BOSON = 1, CTQW_FERMION = 2 } ctqw_statistics;
/* Open chain (N-1 bonds) or ring (N bonds, bond N-1 joins node N-1 to 0). */
typedef enum { CTQW_OPEN = 0, CTQW_PERIODIC = 1 } ctqw_boundary;
/* Interaction energy V(x) added to the diagonal of H:
 *   ONSITE  : U * #{a<b : x_a == x_b}
 *   NEAREST : U * #{a<b : chain distance |x_a - x_b| == 1}                */
typedef enum { CTQW_INT_ONSITE = 0, CTQW_INT_NEAREST = 1 } ctqw_interaction;
/* State precision: interleaved complex FP32 or FP64 (torch.complex64/128). */
typedef enum { CTQW_C64 = 0, CTQW_C128 = 1 } ctqw_dtype;
/* Summation of the Taylor terms within one step.  KAHAN (compensated):
 * the terms Phi^(j), j >= 1, which are smaller than psi by x = dt ||H|| or
 * more, are summed apart from psi and added to it once, so the new state
 * takes one rounding per step (per pass for chained passes) instead of one
 * per term.  PLAIN: each term is added to the running sum as it comes.  The
 * FP64 state always uses PLAIN.                                           */
typedef enum { CTQW_ACC_KAHAN = 0, CTQW_ACC_PLAIN = 1 } ctqw_accumulation;

/* Observables (bit mask).  OCCUPATION: <n_i> = sum_x p(x) #{a : x_a = i},
 * which sums to m.  PAIR: G(i,j) = sum_x p(x) #{a != b : x_a = i, x_b = j}.
 * Both come from the diagonal of the ensemble-averaged density matrix
 * (Eq. 2 and the post-processing stage of Algs. 1-3).                     */
#define CTQW_OBS_OCCUPATION 1u
#define CTQW_OBS_PAIR 2u

typedef struct {
    int32_t m;               /* particles: 1, 2 or 3 (3: distinguishable, equal
                                N_r <= 1024, no gradients)                 */
    int32_t statistics;      /* ctqw_statistics; BOSON needs m == 2 and OPEN */
    int32_t interaction;     /* ctqw_interaction */
    int32_t boundary;        /* ctqw_boundary; PERIODIC needs N >= 3 */
    int32_t dtype;           /* ctqw_dtype */
    int32_t accumulation;    /* ctqw_accumulation (ignored for CTQW_C128) */
    int64_t R;               /* realisations, 1 .. 65535 (UNSUPPORTED above) */
    int32_t n_sites;         /* N for every realisation, or 0 to use ... */
    const int32_t* n_sites_per_real; /* ... [R] sizes (uneven batch), copied */
    double dt;               /* time step, finite and > 0 */
    int32_t taylor_order;    /* > 0: fixed n terms per step (Alg. 3);
                                0: n_r chosen per realisation from taylor_tol;
                                CTQW_RK4_ORDER: the classical Runge-Kutta
                                step of Alg. 2 (see below) */
    double taylor_tol;       /* per-step relative 2-norm truncation tolerance */
    int32_t taylor_max_order;/* cap on n_r; 0 or above the compiled maximum
                                (12 for complex64, 16 for complex128) means
                                that maximum; above it: NOT_CONVERGED */
    int32_t renormalize;     /* 0: monitor the norm only; 1: rescale each step */
    double norm_alarm;       /* |norm - 1| above this -> NUMERICAL; 0: off */
    uint32_t observables;    /* CTQW_OBS_* that ctqw_propagate may be asked for */
} ctqw_problem;

typedef struct ctqw_plan ctqw_plan;

/* Per-step monitoring, FP64 (Alg. 3 "check norm", plus the truncation test). */
typedef struct {
    int64_t steps_done;      /* steps taken since the last ctqw_set_state/init */
    double min_norm;         /* min over realisations of ||psi_r|| after the last step */
    double max_norm;
    double max_tail_ratio;   /* max over r of the estimated truncation error
                                divided by taylor_tol * ||psi_r|| (<= 1 is ok) */
    int32_t min_order, max_order;  /* Taylor terms used per step */
    int64_t alarms;          /* realisation-steps that raised an alarm */
    int32_t flags;           /* bit 0: NOT_CONVERGED, bit 1: NUMERICAL */
} ctqw_step_stats;

/* Launch shape of the propagation kernels.  Defaults are chosen by the
 * library; ctqw_autotune() measures and stores the best one.             */
typedef struct {
    int32_t cols_per_lane;   /* 1 or 2 lattice columns per SIMD lane */
    int32_t waves_per_block; /* 1, 2 or 4 */
    int32_t persistent;      /* 0: one block per group of work items; 1: a grid
                                sized to the device claims groups at run time */
    int32_t use_graph;       /* 1: capture the step loop into a HIP graph */
    int32_t waves_per_cu;    /* persistent grid: resident waves per CU (0: auto) */
    int32_t chunked;         /* 0: all n Taylor terms of a step in one pass over
                                the state when n fits the compiled pipeline
                                (12 terms at one column per lane, 9 complex64
                                / 7 complex128 at two), else passes;
                                1: always passes of K terms (K = 8 complex64,
                                4 complex128, one column per lane), each
                                reading and writing the partial sum and the
                                last term (Alg. 3's term loop split over
                                passes) */
    int32_t band_align;      /* bytes (0, 64, 128 or 256; default 128): the
                                boundaries between the column bands of a
                                realisation are moved down to multiples of
                                this many bytes of a row, so that no cache
                                line of the new state is stored by two waves;
                                per realisation the largest power-of-two
                                fraction of it that needs no more bands than
                                unaligned boundaries is taken (0: bands as
                                wide as the halo allows) */
    int32_t terms_per_pass;  /* three particles: Taylor terms chained per pass
                                over the state, 1..3 (0: 3 for complex64, 2
                                for complex128); a step of n terms is
                                ceil(n / K) passes, the last taking the
                                remaining terms.  Ignored for m < 3.       */
    int32_t band_mode;       /* full grids on open chains, band_align > 0:
                                0 (default): band boundaries on multiples of
                                band_align bytes (above);
                                1: each band's window of columns starts on
                                a multiple of band_align bytes, so its rows
                                are read as whole cache lines, and its
                                output ends on a 32-byte boundary (two bands
                                then store parts of one line).  Other
                                layouts ignore it.                         */
    int32_t three_form;      /* three particles, steps of more than one pass:
                                0 (default): each pass continues the Taylor sum
                                (Eqs. 6-7) from the last term of the one
                                before, carrying the partial sum and that
                                term between passes; the truncation test
                                sees the exact last term;
                                1: product form -- the step's polynomial
                                sum_k z^k / k! (z = -i dt H) factored over its
                                roots, one group of at most terms_per_pass
                                factors per pass, so a pass reads and writes
                                one state; the last term's norm is bounded by
                                (dt G)^(n - K) ||(dt H)^K psi|| from the first
                                pass (G: the Gershgorin bound on ||H||).
                                Ignored for m < 3.                         */
    int32_t row_segments;    /* two particles, all terms in one pass: a band's
                                rows are swept in order by one wave, so a
                                batch with few bands leaves most SIMDs
                                idle.  0 (default): when the batch has
                                fewer than 1024 bands, each band's output
                                rows are split into up to 16 segments
                                (each at least twice the halo long) to
                                bring it to about 1024; 1: never split;
                                2..16: split into up to that many.  A
                                segment is swept from halo rows before its
                                first output row to halo rows after its
                                last (halo = Taylor terms), so the extra
                                reads are 2 * halo rows per segment.       */
} ctqw_launch;

/* Create a plan from a problem statement.  Host only: validates the
 * problem, computes the state layout.  No device is touched.
 * Errors: INVALID_ARG (NULL, m not in 1..3, N < 2, periodic with N < 3,
 * non-finite or non-positive dt, order and tol both unset, bad enums),
 * UNSUPPORTED (m == 3 unless distinguishable with one lattice size
 * N <= 1024; bosons or fermions with m != 2 or on a ring; R > 65535),
 * OUT_OF_MEMORY.                                                           */
ctqw_status ctqw_plan_create(const ctqw_problem* problem, ctqw_plan** out);
ctqw_status ctqw_plan_destroy(ctqw_plan* plan);

/* Static parameters of every realisation (Eq. 1 with the noise drawn):
 * J   : packed per realisation, n_bonds(N_r) values each (N_r - 1 open,
 *       N_r periodic); bond i joins node i and node i+1 (mod N_r).
 * eps : packed per realisation, N_r on-site energies each.
 * U   : [R] interaction strengths.
 * Realisations are packed in order r = 0..R-1.  Copied.  Computes the
 * Taylor order n_r of each realisation (see ctqw_orders).
 * Errors: INVALID_ARG (NULL, non-finite), NOT_CONVERGED (n_r above cap).   */
ctqw_status ctqw_set_params(ctqw_plan* plan, const double* J, const double* eps,
                            const double* U);
ctqw_status ctqw_get_params(const ctqw_plan* plan, double* J, double* eps, double* U);

/* Noise model of Eq. 1 with static draws: parameter = baseline + draw,
 * independent across realisations (the paper draws noise on the hoppings;
 * on-site and interaction noise follow the same form).                   */
typedef enum { CTQW_DIST_NONE = 0, CTQW_DIST_UNIFORM = 1 /* U[a, b] */,
               CTQW_DIST_NORMAL = 2 /* N(a, b^2) */ } ctqw_dist;
typedef struct {
    int32_t dist;            /* ctqw_dist */
    double a, b;
} ctqw_noise;

/* Draw every realisation's parameters on the host and apply them as
 * ctqw_set_params does.  J_base: [n_bonds(max N_r)] baseline hoppings, or
 * NULL for 1 on every bond; eps_base: [max N_r] baseline energies, or NULL
 * for 0; realisation r uses the first n_bonds(N_r) / N_r entries.  A NULL
 * noise pointer means no noise.  Generator: Philox4x32-10 (Salmon et al.,
 * SC 2011), one block per parameter with counter (index, kind, r mod 2^32,
 * r div 2^32) -- kind 0 bonds, 1 sites, 2 interaction -- and key (seed mod
 * 2^32, seed div 2^32); from the block (w0..w3), u = (2^26 (w0 >> 5) +
 * (w1 >> 6)) 2^-53 and v likewise from (w2, w3); uniform: a + (b - a) u;
 * normal: a + b sqrt(-2 log(1 - u)) cos(2 pi v), in double without fused
 * operations.  The drawn values are returned by ctqw_get_params.
 * Errors: as ctqw_set_params; INVALID_ARG for an unknown dist or a
 * non-finite a, b or baseline.                                            */
ctqw_status ctqw_draw_params(ctqw_plan* plan, const double* J_base, const double* eps_base, double U_base,
                             const ctqw_noise* J_noise, const ctqw_noise* eps_noise, const ctqw_noise* U_noise,
                             uint64_t seed);

/* Alg. 2 (classical fourth-order Runge-Kutta).  For dpsi/dt = -i H psi
 * with H constant over the step, the stages K1 = A psi, K2 = A (psi +
 * K1/2), K3 = A (psi + K2/2), K4 = A (psi + K3) with A = -i dt H combine
 * to psi + (K1 + 2 K2 + 2 K3 + K4)/6 = sum_{k<=4} A^k psi / k!, the
 * degree-4 Taylor step; taylor_order = CTQW_RK4_ORDER (with taylor_tol
 * unused) therefore runs Alg. 2, as one fused pass per step.  Like any
 * truncated series it does not conserve the norm exactly.                 */
#define CTQW_RK4_ORDER 4

/* Time-dependent hopping noise (Eq. 1 with switching stochastic terms):
 * every bond i of every realisation r carries J_i(t) = Jbar_i + xi_i(t)
 * with Jbar the J of ctqw_set_params and xi = +-amplitude, flipping sign at
 * the events of a Poisson process of the given rate (per unit time).  At
 * the start of step s each bond flips with probability 1 - exp(-rate dt)
 * and the new J holds during the step.  Draws: Philox4x32-10, counter
 * (i, 4 (s + 1), r mod 2^32, r div 2^32), key (seed mod 2^32 XOR
 * 0x54454C45, seed div 2^32), u = 53-bit fraction of (w0, w1): flip if
 * u < p; s = -1 gives the initial sign, + if u < 1/2.  The a-priori
 * orders take |Jbar_i| + amplitude.  The process starts (s = 0) whenever
 * the tables are uploaded — the first device call after this one,
 * ctqw_set_params, ctqw_set_launch or a re-bind — and advances one draw
 * per step, also inside captured step loops.
 * amplitude = 0 returns to static noise.  Not combined with gradients.
 * Errors: INVALID_ARG (negative or non-finite), NOT_CONVERGED (orders). */
ctqw_status ctqw_set_telegraph(ctqw_plan* plan, double amplitude, double rate, uint64_t seed);

/* Taylor terms per step of each realisation, [R].  With taylor_order > 0
 * every entry is taylor_order; otherwise n_r is the smallest n >= 1 with
 * x^(n+1)/(n+1)! / (1 - x/(n+2)) <= taylor_tol, x = dt * G_r, where G_r =
 * m * max_i(|eps_i| + |J_(i-1)| + |J_i|) + |U_r| m(m-1)/2 bounds ||H_r||_2
 * (Gershgorin).  Valid after ctqw_set_params.
 * Steps of one and two particles apply each realisation's own n_r: items
 * are grouped by order and each group is one launch at that depth.  The
 * batch's largest order is applied to every realisation by chunked passes,
 * by three-particle steps, and in ctqw_gradient (one polynomial for the
 * adjoint); the truncation estimate follows the order applied.           */
ctqw_status ctqw_orders(const ctqw_plan* plan, int32_t* orders);

/* Amplitudes stored per realisation and their offsets in a state buffer.
 * Layouts (interleaved complex, re then im):
 *   m = 1                : psi[x], N_r amplitudes.
 *   m = 2 distinguishable: psi[x1][x2], x2 fastest, N_r^2 amplitudes.
 *   m = 2 bosons         : the exchange-symmetric amplitude phi(x1, x2)
 *                          for x1 <= x2, row-major (row x1 holds x2 = x1..N-1),
 *                          N_r (N_r + 1) / 2 amplitudes.  In the normalised
 *                          symmetric basis the coefficient of |x1 x2> is
 *                          sqrt(2) phi for x1 < x2 and phi for x1 == x2.
 *   m = 3 distinguishable: psi[x1][x2][x3], x3 fastest, N_r^3 amplitudes.
 * offsets: [R + 1], in amplitudes; offsets[R] is the total.                */
ctqw_status ctqw_layout(const ctqw_plan* plan, int64_t* offsets);

/* One particle on a general graph (Sec. 2: each node couples to its own
 * set of neighbours; a q-dimensional lattice, q > 1, is one such graph), R
 * statically noisy realisations sharing one topology, advanced n_steps
 * times by the order-n Taylor polynomial of exp(-i H dt) (Eqs. 5-7), one
 * pass over the batch per term.  Two particles on a graph are one particle
 * on the pair graph (ctqw_graph_tables builds its tables: distinguishable,
 * boson or fermion pairs; a fermion move that flips the pair's order carries
 * a negative weight, so hop values may take either sign).  Stateless: no plan.
 * dtype CTQW_C128: complex128 states, FP64 tables and arithmetic;
 * CTQW_C64: complex64 states, FP32 tables and arithmetic, plain sums.
 *   nbr     device int32 [width][n_nodes]: neighbour of node i in slot k is
 *           nbr[k * n_nodes + i]; a value outside [0, n_nodes) (use -1)
 *           marks an empty slot, so nodes may have different degrees.
 *   hop     device real [R][width][n_nodes]: H_r[i, nbr[k][i]] =
 *           hop[(r * width + k) * n_nodes + i].  H_r is Hermitian only if
 *           the caller gives both directions of every bond the same value
 *           (not checked).  nbr and hop may be NULL when width == 0.
 *   onsite  device real [R][n_nodes]: H_r[i, i].
 *   psi     device complex [R][n_nodes] (interleaved re, im), advanced in
 *           place.
 *   workspace  device memory of ctqw_graph_workspace(n_nodes, R, dtype)
 *           bytes.
 *   norms   device double [n_steps][R] or NULL: the squared FP64 2-norm
 *           of each realisation after each step (the per-step norm check
 *           of Alg. 3; a fixed summation order, so reruns give the same
 *           bits).  The library raises no alarm on this path: the caller
 *           reads the norms.
 * order: 1..64 terms (fixed).  Enqueued on hip_stream (hipStream_t, NULL =
 * default); psi, the tables and the workspace must stay valid until the
 * work has run.  Errors: INVALID_ARG (non-positive sizes, unknown dtype,
 * NULL, non-finite dt, order out of range, workspace too small), DEVICE.  */
/* Tables of ctqw_graph_evolve from an undirected bond list (Sec. 2: each
 * node couples to its own neighbours; Eq. 1 with equal rates both ways),
 * built on the host.  edges: int32 [n_edges][2] node pairs (no self-loops,
 * no repeated bonds); J: [R][n_edges] bond couplings, eps: [R][n_nodes]
 * on-site energies, U: [R] on-site interaction (m == 2; NULL for m == 1).
 *   m = 1: states are the nodes; every bond fills one slot of both of its
 *          nodes, in bond order (first endpoint first); width = the
 *          largest degree.
 *   m = 2: one particle on the pair graph.  States: ordered pairs (a, b) at
 *          a * n + b (DISTINGUISHABLE); pairs a <= b in lexicographic order,
 *          each the normalised symmetric state (BOSON); pairs a < b, each the
 *          normalised antisymmetric state (FERMION).  Either particle moves
 *          along one of its node's slots (width = 2 x the one-particle
 *          width: slots of the first particle, then of the second).  Bosons:
 *          a move between (a, a) and (a, c) carries sqrt(2) J, split as
 *          J / sqrt(2) over the two slots of the diagonal state.  Fermions: a
 *          move onto the other particle's node is absent, and one that
 *          carries the mover past the other particle (the pair's order
 *          flips) carries -J.  On-site energies add; U sits on the states
 *          with both particles on one node (none for fermions).
 * Outputs (host, caller-allocated): n_states, width; then, unless nbr, hop
 * and onsite are all NULL (a size query), nbr int32 [width][n_states] (-1
 * in empty slots), hop double [R][width][n_states] (0 in empty slots),
 * onsite double [R][n_states].  Errors: INVALID_ARG (sizes, NULL, a node
 * out of range, self-loop, repeated bond, non-finite parameter),
 * UNSUPPORTED (tables beyond 2^31 entries).                               */
ctqw_status ctqw_graph_tables(int32_t n_nodes, int32_t n_edges, const int32_t* edges, int32_t m, int32_t statistics,
                              int32_t R, const double* J, const double* eps, const double* U, int32_t* n_states,
                              int32_t* width, int32_t* nbr, double* hop, double* onsite);

/* A-priori Taylor orders for ctqw_graph_evolve, computed on the host from
 * host copies of its tables (same layouts, FP64): orders[r] is the smallest
 * n >= 1 with x^(n+1)/(n+1)! / (1 - x/(n+2)) <= tol, x = |dt| * G_r and
 * G_r = max_i (|onsite_r[i]| + sum over filled slots |hop_r[k][i]|), the
 * Gershgorin bound on ||H_r||_2 (the chain path's rule, Alg. 3's order
 * chosen before the step).  Errors: INVALID_ARG, NOT_CONVERGED (a
 * realisation needs more than max_order <= 64 terms).                    */
ctqw_status ctqw_graph_orders(int32_t n_nodes, int32_t width, const int32_t* nbr, const double* hop,
                              const double* onsite, int32_t R, double dt, double tol, int32_t max_order,
                              int32_t* orders);
ctqw_status ctqw_graph_workspace(int32_t n_nodes, int32_t R, int32_t dtype, int64_t* bytes);
ctqw_status ctqw_graph_evolve(int32_t n_nodes, int32_t width, const int32_t* nbr, const void* hop,
                              const void* onsite, int32_t R, int32_t dtype, double dt, int32_t order,
                              int64_t n_steps, void* psi, void* workspace, int64_t workspace_bytes,
                              double* norms, void* hip_stream);

/* One particle on a two-dimensional lattice (q = 2, Sec. 2; the capacity
 * example of Sec. 3) with every bond and node of every realisation carrying
 * its own coupling and on-site energy (Eq. 1 with the noise drawn per bond
 * and per node), advanced by the truncated Taylor series of exp(-i H dt)
 * (Eqs. 5-7, Alg. 3): all `order` terms of a step are chained in one pass
 * over the state (a register pipeline down the rows, 64-column bands with
 * a halo of `order` columns), where ctqw_graph_evolve runs one pass per
 * term.  The node (x, y) of realisation r is element r * Lx * Ly + y * Lx
 * + x of every array (the node numbering of a row-major lattice).
 *   Lx, Ly       lattice size (>= 1); periodic_x / periodic_y: 1 closes the
 *                axis into a ring (of at least 3 nodes), 0 leaves it open
 *   Jx, Jy, eps  device arrays [R][Ly][Lx] of the state's real type
 *                (float for CTQW_C64, double for CTQW_C128): the coupling
 *                between (x, y) and (x + 1, y), between (x, y) and
 *                (x, y + 1) (ignored at an open axis's last column / row),
 *                and the on-site energy; read only
 *   psi          device state [R][Ly][Lx], complex, updated in place
 *   workspace    ctqw_lattice_workspace bytes of device memory, 256-byte
 *                aligned (a second state buffer, the dt-scaled tables and
 *                the norm partials)
 *   norms        device double [n_steps][R] or NULL: the squared FP64
 *                2-norm of each realisation after each step (per band in a
 *                fixed order, then over the bands in band order)
 * order: 1..12 (complex64) or 1..10 (complex128); a larger order is
 * UNSUPPORTED here (ctqw_graph_evolve takes up to 64).  Enqueued on
 * hip_stream (NULL = default); the call does not synchronise.  Errors:
 * INVALID_ARG (sizes, NULL, non-finite dt, workspace too small or
 * misaligned), UNSUPPORTED (order, tables beyond 2^31 entries), DEVICE. */
ctqw_status ctqw_lattice_workspace(int32_t Lx, int32_t Ly, int32_t R, int32_t dtype, int32_t order,
                                   int32_t periodic_x, int64_t* bytes);
ctqw_status ctqw_lattice_evolve(int32_t Lx, int32_t Ly, int32_t periodic_x, int32_t periodic_y, int32_t R,
                                const void* Jx, const void* Jy, const void* eps, int32_t dtype, double dt,
                                int32_t order, int64_t n_steps, void* psi, void* workspace,
                                int64_t workspace_bytes, double* norms, void* hip_stream);

/* ctqw_graph_evolve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments and kernels without the workspace, whose
 * role -- two term buffers and the partial sum, ctqw_graph_workspace bytes
 * -- is taken by a fixed array of CTQW_GRAPH_STATIC_BYTES in device memory
 * that the library holds on each device it runs on until the process
 * ends.  The call allocates nothing (no hipMalloc, no allocating library
 * routine).  Every call on one device shares that device's array, so
 * calls that overlap on one device (other streams, other host threads)
 * race; the caller serialises them.  The stream's device (the current
 * device for the NULL stream) is the one used.
 * Errors: as ctqw_graph_evolve; UNSUPPORTED (checked before any device
 * call) when ctqw_graph_workspace(n_nodes, R, dtype) exceeds
 * CTQW_GRAPH_STATIC_BYTES; DEVICE if the array's address cannot be found. */
#define CTQW_GRAPH_STATIC_BYTES (64ll << 20)
ctqw_status ctqw_graph_evolve_static(int32_t n_nodes, int32_t width, const int32_t* nbr, const void* hop,
                                     const void* onsite, int32_t R, int32_t dtype, double dt, int32_t order,
                                     int64_t n_steps, void* psi, double* norms, void* hip_stream);

/* Device bytes the caller must provide: each of the two state buffers and
 * the workspace, for the current parameters and launch shape.             */
ctqw_status ctqw_sizes(const ctqw_plan* plan, int64_t* state_bytes, int64_t* workspace_bytes);

/* Bind caller-owned device memory and a HIP stream (hipStream_t, may be
 * NULL for the default stream) and upload the parameter tables.  psi_a and
 * psi_b are the ping-pong state buffers.  The buffers must stay valid
 * until the plan is destroyed or re-bound.  Errors: INVALID_ARG (NULL or a
 * buffer smaller than ctqw_sizes), STATE (params not set), DEVICE.        */
ctqw_status ctqw_bind(ctqw_plan* plan, void* psi_a, void* psi_b, int64_t state_bytes,
                      void* workspace, int64_t workspace_bytes, void* hip_stream);

/* Start state: particle a on node sites[a] (per_realization == 0, [m]
 * entries) or sites[r*m + a] (per_realization == 1, [R*m]).  Bosons get the
 * normalised symmetric state of that occupation.  Resets steps_done.
 * Errors: INVALID_ARG (site out of range), STATE (not bound).             */
ctqw_status ctqw_init_product_state(ctqw_plan* plan, const int32_t* sites, int32_t per_realization);

/* Copy the whole current state (layout of ctqw_layout, dtype of the plan)
 * in or out.  on_device != 0: psi is a device pointer; else host memory.   */
ctqw_status ctqw_set_state(ctqw_plan* plan, const void* psi, int32_t on_device);
ctqw_status ctqw_get_state(ctqw_plan* plan, void* psi, int32_t on_device);

/* Advance every realisation by n_steps steps of Alg. 3.  If output_every
 * > 0 and obs != 0, the ensemble observables are evaluated at step 0 and
 * after every output_every steps and written to out (host, FP64):
 *   n_out = n_steps / output_every + 1 snapshots, groups = distinct lattice
 *   sizes in ascending order, and for each snapshot and group
 *     OCCUPATION: N_g values, then PAIR: N_g * N_g values (row-major),
 *   snapshot-major: [n_out][group][OCC block then PAIR block].
 * Errors: STATE, INVALID_ARG (obs not enabled in the problem),
 * NOT_CONVERGED / NUMERICAL (alarms raised during the run), DEVICE.       */
ctqw_status ctqw_propagate(ctqw_plan* plan, int64_t n_steps, int64_t output_every,
                           uint32_t obs, double* out);

/* Ensemble observables of the current state, same layout as one snapshot. */
ctqw_status ctqw_observe(ctqw_plan* plan, uint32_t obs, double* out);

/* Number of groups (distinct lattice sizes) and their sizes, ascending.   */
ctqw_status ctqw_groups(const ctqw_plan* plan, int32_t* n_groups, int32_t* sizes);

/* Ensemble-averaged density matrix of one group (Eq. 2; the paper updates
 * it with one Hermitian rank-1 update per realisation):
 *     rho_g = (1/R_g) sum_{r in g} |psi_r><psi_r|,
 * D_g x D_g complex of the plan's dtype in the basis of ctqw_layout (bosons
 * and fermions: the triangle basis, coefficient sqrt(2) phi off the
 * diagonal; the fermions' diagonal rows and columns are zero), column-major
 * with leading dimension ld >= D_g, written to the caller's device memory
 * rho.  lower_only != 0: only the lower triangle is written (the upper one
 * is left as it was); else the full Hermitian matrix.  workspace: device
 * memory of at least ctqw_density_workspace(group) bytes, which receives
 * the group's states (load scale and basis weights applied) as real and
 * imaginary planes padded with zeros to whole tiles (128 rows complex64, 64
 * complex128) and stages (16 / 8 realisations); the lower triangle of
 * rho = A A^H / R_g is then formed tile by tile on the matrix cores
 * (FP32 MFMA for complex64, FP64 MFMA for complex128).  Enqueued on the
 * plan's stream.  Errors: INVALID_ARG (NULL, group out of range, ld or
 * workspace too small), UNSUPPORTED (D_g or ld >= 2^31, R_g > 65535),
 * STATE (not bound), DEVICE.                                              */
ctqw_status ctqw_density_workspace(const ctqw_plan* plan, int32_t group, int64_t* bytes);
ctqw_status ctqw_density_matrix(ctqw_plan* plan, int32_t group, void* rho, int64_t ld, int32_t lower_only,
                                void* workspace, int64_t workspace_bytes);

/* Monitoring after the last step (see ctqw_step_stats).                   */
ctqw_status ctqw_stats(ctqw_plan* plan, ctqw_step_stats* out);
/* FP64 squared norms and estimated squared truncation errors of every
 * realisation after the last step, [R] each (either may be NULL).         */
ctqw_status ctqw_realization_norms(ctqw_plan* plan, double* norm2, double* tail2);

/* Launch shape (see ctqw_launch).  Setting it may change ctqw_sizes.      */
ctqw_status ctqw_get_launch(const ctqw_plan* plan, ctqw_launch* out);
ctqw_status ctqw_set_launch(ctqw_plan* plan, const ctqw_launch* launch);

/* Number of work items (realisation x column band, or row segment of a
 * band) of one step and the number of waves that one step launches, for
 * the current launch shape (regular: whole blocks of waves_per_block
 * waves; persistent: the device's resident waves, known once bound; with
 * several orders, the largest of the per-order launches).                */
ctqw_status ctqw_work_items(const ctqw_plan* plan, int64_t* items, int64_t* waves);

/* Derivatives of an ensemble-averaged diagonal observable.  The paper does
 * not differentiate; this extends its method.  With the state at the call
 * as psi_0 and T = n_steps steps of Alg. 3 (the same map ctqw_propagate
 * applies), the loss is
 *     L = (1/R) sum_r <psi_r(T)| W |psi_r(T)>,  W diagonal in the occupation basis,
 *   ONE_BODY: w(x) = sum_a g[x_a];   PRODUCT: w(x) = prod_a g[x_a]
 * (g = site_weights[N]; PRODUCT with g the indicator of a block of nodes is
 * the probability that all particles are in it).  The noise is additive
 * (J^r = Jbar + dJ^r, eps^r = epsbar + deps^r), so dL/dJbar_i =
 * sum_r dL/dJ^r_i; grad_J [n_bonds(N)] and grad_eps [N] return these, the
 * exact derivatives of the discrete (truncated-Taylor) map, computed by a
 * hand-written adjoint: the forward run keeps the state every ckpt_every
 * steps, each segment is recomputed from its checkpoint, and the adjoint of
 * every step applies p(A)^dagger with A = -i dt H by a Horner recursion
 * (the same stencil with dt -> -dt) while FP64 kernels contract the bond
 * and site operators.  All realisations must share one lattice size, whose
 * state is under 2^31 bytes (two particles: N <= 16383 complex64, 11585
 * complex128; UNSUPPORTED above); renormalize must be 0.  grad_ws is
 * caller-owned device memory of at
 * least ctqw_gradient_workspace bytes (256-byte aligned).  On return the
 * current state is psi(T).                                                */
#define CTQW_LOSS_ONE_BODY 0
#define CTQW_LOSS_PRODUCT 1
ctqw_status ctqw_gradient_workspace(const ctqw_plan* plan, int64_t n_steps, int64_t ckpt_every, int64_t* bytes);
/* The two halves of ctqw_gradient: ctqw_forward_ckpt advances n_steps and
 * keeps the checkpoints in grad_ws; ctqw_backward evaluates the loss at the
 * current state and runs the adjoint back to the state the forward started
 * from.  Changing parameters, launch shape or state in between invalidates
 * the checkpoints (CTQW_ERR_STATE); one backward per forward.            */
ctqw_status ctqw_forward_ckpt(ctqw_plan* plan, int64_t n_steps, int64_t ckpt_every, void* grad_ws,
                              int64_t grad_ws_bytes);
ctqw_status ctqw_backward(ctqw_plan* plan, int32_t kind, const double* site_weights, void* grad_ws,
                          int64_t grad_ws_bytes, double* loss, double* grad_J, double* grad_eps);
/* The loss alone at the current state (FP64).  Uses scratch at the end of
 * grad_ws (at least ctqw_gradient_workspace(plan, 0, 1) bytes) and leaves
 * the checkpoints of a pending ctqw_forward_ckpt intact.                  */
ctqw_status ctqw_loss(ctqw_plan* plan, int32_t kind, const double* site_weights, void* grad_ws,
                      int64_t grad_ws_bytes, double* loss);
ctqw_status ctqw_gradient(ctqw_plan* plan, int64_t n_steps, int64_t ckpt_every, int32_t kind,
                          const double* site_weights, void* grad_ws, int64_t grad_ws_bytes, double* loss,
                          double* grad_J, double* grad_eps);

/* Autotuner.  Times `steps` propagation steps (after one warm-up step) for
 * every launch shape -- columns per lane {1, 2}, waves per block {1, 2, 4},
 * regular or persistent launch, for the persistent form a cap of
 * {auto, 8, 16} resident waves per CU, all terms in one pass or passes of
 * K terms (one column per lane), band alignment {128, 64, 0} bytes and
 * band layout (output- or window-aligned); for three particles the terms
 * per pass {3, 2, 1} and the x3 band alignment -- that fits the bound workspace,
 * keeps the fastest (average step-kernel time from HIP events) and applies
 * it with ctqw_set_launch (use_graph is left as set).  With a cache path
 * (or the CTQW_TUNE_CACHE environment variable when cache_path is NULL),
 * a stored result for the same device, library version and problem shape
 * (dtype, accumulation, m, statistics, boundary, lattice sizes, R, Taylor
 * orders) is applied without timing, and new results are appended (one
 * JSON object per line).  If the CTQW_TUNE_TRACE environment variable
 * names a file, one line per candidate (its shape and time, or that it does
 * not fit the bound workspace) is appended to it.  The state buffers are
 * overwritten: tune before ctqw_init_product_state / ctqw_set_state.
 * best / best_ms may be NULL.                                              */
ctqw_status ctqw_autotune(ctqw_plan* plan, const char* cache_path, int32_t steps, ctqw_launch* best,
                          double* best_ms);

/* Kernel timing: with enable != 0, every step-kernel launch is bracketed by
 * HIP events on the bound stream and ctqw_get_timing returns the summed
 * elapsed time (ms) and the number of timed steps since timing was
 * (re-)enabled.  With use_graph the events bracket each replay of a captured
 * step loop, which counts for its steps: the time then also holds the FP64
 * finalize kernel of each step.  For measurement only.                    */
ctqw_status ctqw_set_timing(ctqw_plan* plan, int32_t enable);
ctqw_status ctqw_get_timing(ctqw_plan* plan, double* step_kernel_ms, int64_t* launches);

/* Memory-bandwidth probes, for reading the kernels' rates against what the
 * memory system sustains (measurement only; no part of the method runs).
 *   pattern 0: copy `bytes` from src to dst, one 16-byte element per thread
 *              (the fastest plain copy form found on gfx950); n and
 *              waves_per_cu are ignored.
 *   pattern 1: the access pattern of the two-particle step kernel with its
 *              arithmetic taken out: src and dst hold bytes / (8 n^2) grids
 *              of n x n complex64 (rows of 8n bytes, n a multiple of 128),
 *              and one wave per band of 128 columns (1 KiB of a row) copies
 *              its band row by row with two rows of loads in flight, at most
 *              waves_per_cu resident waves per CU (4..32; 0: 8, the step
 *              kernel's occupancy at two columns per lane).
 * src and dst are device buffers of `bytes` bytes that do not overlap;
 * bytes is a multiple of 16 (pattern 0) or of 8 n^2 (pattern 1).
 * Enqueued on hip_stream (hipStream_t, NULL = default); does not
 * synchronise.  Errors: INVALID_ARG (NULL, overlap, sizes, pattern),
 * DEVICE (launch failed).                                                  */
ctqw_status ctqw_bandwidth_probe(const void* src, void* dst, int64_t bytes, int32_t pattern, int32_t n,
                                 int32_t waves_per_cu, void* hip_stream);

const char* ctqw_status_string(ctqw_status status);
const char* ctqw_last_error(const ctqw_plan* plan);
/* Library version string. */
const char* ctqw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CTQW_H */
