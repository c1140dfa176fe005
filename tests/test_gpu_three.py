"""GPU parity for three distinguishable walkers (K Taylor terms chained per
pass over the state, K = 1, 2, 3, the last pass taking the remaining
terms): against the oracle's exact evolution on small lattices, against
its Taylor map on lattices that span several tiles in both plane
directions, on the three-walker workload's parameters for one output
interval, and on the full N = 256 lattice against the oracle on the window
the walkers can reach."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import hamiltonian as Hm
from oracle import observables as O
from oracle import propagate as P
from workloads import C5, scaled

from _helpers import gpu_plan, say

pytestmark = pytest.mark.gpu


def reals3(N, R, seed, boundary="open"):
    g = np.random.default_rng(seed)
    nb = N if boundary == "periodic" else N - 1
    return [(N, 1 + 0.2 * g.standard_normal(nb), g.uniform(-1, 1, N), float(g.uniform(0.5, 1.5))) for _ in range(R)]


@pytest.mark.parametrize("K", [1, 2, 3])
@pytest.mark.parametrize("N,boundary,interaction", [(7, "open", "nearest"), (10, "open", "nearest"),
                                                    (6, "periodic", "onsite"), (5, "periodic", "nearest")])
def test_three_walkers_c128_against_ed(N, boundary, interaction, K):
    say(f"case: m=3 N={N} {boundary} {interaction} c128, K={K}, 40 steps")
    R, dt, steps = 3, 0.02, 40
    reals = reals3(N, R, 1, boundary)
    sites = [1, N // 2, N - 2]
    plan = gpu_plan(m=3, statistics="distinguishable", boundary=boundary, interaction=interaction, dtype="c128",
                    reals=reals, dt=dt, tol=1e-14, observables=3, sites=sites, launch={"terms_per_pass": K})
    out = plan.propagate(steps, 20, 3)
    psi = plan.state_numpy()
    st = B.basis_states(N, 3)
    worst, occ, pair = 0.0, [], []
    for r, (n, J, eps, U) in enumerate(reals):
        H = Hm.hamiltonian(N, 3, J, eps, U, B.DISTINGUISHABLE, boundary, interaction)
        ref = P.EDPropagator(H).evolve(B.product_state(N, sites), dt * steps)
        worst = max(worst, float(np.max(np.abs(psi[r * N ** 3:(r + 1) * N ** 3] - ref))))
        occ.append(O.occupation(ref, st, N))
        pair.append(O.pair_correlation(ref, st, N))
    occ_e, pair_e = O.ensemble_mean(occ), O.ensemble_mean(pair)
    e_occ = np.max(np.abs(out[-1][:N] - occ_e))
    e_pair = np.max(np.abs(out[-1][N:].reshape(N, N) - pair_e))
    n2, _ = plan.realization_norms()
    say(f"  order {int(plan.orders().max())}: amplitude {worst:.2e}, occupation {e_occ:.2e}, pair {e_pair:.2e}, "
        f"|norm^2 - 1| {np.max(np.abs(n2 - 1)):.1e}")
    assert worst <= 1e-10 and e_occ <= 1e-10 and e_pair <= 1e-10
    assert abs(out[0][:N].sum() - 3) < 1e-12
    assert np.max(np.abs(n2 - 1)) < 1e-12


@pytest.mark.parametrize("N,boundary,K", [(70, "open", 3), (41, "open", 2), (37, "periodic", 3)])
def test_three_walkers_several_tiles_c128(N, boundary, K):
    """Lattices spanning several tiles along x2 and x3 (a tile is 64 x3
    columns by 16-24 x2 rows at complex128) with a ragged last tile: the
    state after 12 steps equals the oracle's Taylor map of the same order,
    amplitude by amplitude (1e-12), from a random complex start state; the
    FP64 norms follow the oracle's."""
    R, dt, steps = 2, 0.02, 12
    reals = reals3(N, R, 7, boundary)
    say(f"case: m=3 several tiles N={N} {boundary} K={K} c128, {steps} steps")
    g = np.random.default_rng(11)
    D = N ** 3
    psi0 = g.standard_normal((R, D)) + 1j * g.standard_normal((R, D))
    psi0 /= np.linalg.norm(psi0, axis=1, keepdims=True)
    plan = gpu_plan(m=3, statistics="distinguishable", boundary=boundary, interaction="nearest", dtype="c128",
                    reals=reals, dt=dt, tol=1e-14, launch={"terms_per_pass": K})
    plan.set_state_numpy(psi0.reshape(-1))
    n = int(plan.orders().max())
    plan.propagate(steps)
    psi = plan.state_numpy().reshape(R, D)
    n2, _ = plan.realization_norms()
    worst = 0.0
    for r, (_, J, eps, U) in enumerate(reals):
        H = Hm.hamiltonian(N, 3, J, eps, U, B.DISTINGUISHABLE, boundary, "nearest")
        ref, _, _ = P.evolve_taylor(H, psi0[r], dt, steps, order=n)
        worst = max(worst, float(np.max(np.abs(psi[r] - ref))))
        assert abs(n2[r] - np.vdot(ref, ref).real) < 1e-12
    say(f"  order {n}: max |psi - oracle map| = {worst:.2e}")
    assert worst <= 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("K", [1, 2, 3])
def test_three_walkers_middle_passes_every_lane(K, dtype):
    """One step of order 3K (a first, a middle and a last pass) on a 70-site
    chain whose tiles hold amplitudes in all 64 lanes and all rows: every
    amplitude equals the oracle's Taylor map of that order (complex128
    1e-12; complex64 5e-9 on amplitudes of size ~1e-3).  A middle pass both
    reads the partial sum and writes the next pass's seed; a store whose
    data registers were overwritten before it read them once showed up here
    as wrong real parts in four-lane groups."""
    N, dt, order = 70, 0.02, 3 * K
    reals = reals3(N, 1, 7, "open")
    say(f"case: m=3 middle passes N={N} K={K} order={order} {dtype}")
    g = np.random.default_rng(11)
    D = N ** 3
    psi0 = g.standard_normal(D) + 1j * g.standard_normal(D)
    psi0 /= np.linalg.norm(psi0)
    plan = gpu_plan(m=3, statistics="distinguishable", boundary="open", interaction="nearest", dtype=dtype,
                    reals=reals, dt=dt, order=order, launch={"terms_per_pass": K})
    plan.set_state_numpy(psi0)
    plan.propagate(1)
    psi = plan.state_numpy()
    _, J, eps, U = reals[0]
    H = Hm.hamiltonian(N, 3, J, eps, U, B.DISTINGUISHABLE, "open", "nearest")
    ref, _, _ = P.evolve_taylor(H, psi0, dt, 1, order=order)
    err = np.abs(psi - ref)
    say(f"  max |psi - oracle map| = {err.max():.2e}, entries above the bar: "
        f"{int((err > (1e-12 if dtype == 'c128' else 5e-9)).sum())}")
    assert err.max() <= (1e-12 if dtype == "c128" else 5e-9)


def test_three_walker_workload_one_output_interval_c64():
    """The three-walker workload's parameters (nearest-neighbour U = 1,
    eps ~ U[-1, 1], J = 1, dt = 0.02, tolerance 1e-7, complex64, start at the
    centre) on a reduced lattice N = 48, for one output interval of 50 steps,
    against the oracle's exact evolution: amplitudes within 2e-6, ensemble
    occupation and pair correlation within 1e-6, norms within 1e-6."""
    w = scaled(C5(), N=48, R=3, start=(23, 24, 25))
    reals = w.all_realizations()
    steps = 50
    say(f"case: {w.name} reduced to N=48 R=3, {steps} steps c64")
    plan = gpu_plan(m=3, statistics="distinguishable", boundary="open", interaction="nearest", dtype="c64",
                    reals=reals, dt=w.dt, tol=w.tol, observables=3, sites=list(w.start))
    out = plan.propagate(steps, steps, 3)
    psi = plan.state_numpy()
    st = B.basis_states(w.N, 3)
    worst, occ, pair = 0.0, [], []
    D = w.N ** 3
    for r, (N, J, eps, U) in enumerate(reals):
        H = Hm.hamiltonian(N, 3, J, eps, U, B.DISTINGUISHABLE, "open", "nearest")
        ref, _, _ = P.evolve_taylor(H, B.product_state(N, list(w.start)), w.dt, steps, tol=1e-15)
        worst = max(worst, float(np.max(np.abs(psi[r * D:(r + 1) * D] - ref))))
        occ.append(O.occupation(ref, st, N))
        pair.append(O.pair_correlation(ref, st, N))
    e_occ = float(np.max(np.abs(out[-1][:w.N] - O.ensemble_mean(occ))))
    e_pair = float(np.max(np.abs(out[-1][w.N:].reshape(w.N, w.N) - O.ensemble_mean(pair))))
    n2, _ = plan.realization_norms()
    say(f"  order {int(plan.orders().max())}: amplitude {worst:.2e}, occupation {e_occ:.2e}, pair {e_pair:.2e}, "
        f"|norm - 1| {np.max(np.abs(np.sqrt(n2) - 1)):.1e}")
    assert worst <= 2e-6 and e_occ <= 1e-6 and e_pair <= 1e-6
    assert np.max(np.abs(np.sqrt(n2) - 1)) <= 1e-6


def test_three_walker_autotune_picks_a_pass_depth():
    """The autotuner times 1, 2 and 3 terms per pass for three walkers and
    applies the fastest; the tuned plan still matches the oracle."""
    N, R, dt, steps = 9, 2, 0.02, 10
    reals = reals3(N, R, 5)
    sites = [2, 4, 6]
    say("case: m=3 autotune N=9 c128")
    plan = gpu_plan(m=3, statistics="distinguishable", boundary="open", interaction="nearest", dtype="c128",
                    reals=reals, dt=dt, tol=1e-14)
    best, ms = plan.autotune(steps=2)
    assert best.terms_per_pass in (1, 2, 3) and ms > 0
    plan.init_product_state(sites)
    plan.propagate(steps)
    psi = plan.state_numpy()
    for r, (n, J, eps, U) in enumerate(reals):
        H = Hm.hamiltonian(N, 3, J, eps, U, B.DISTINGUISHABLE, "open", "nearest")
        ref = P.EDPropagator(H).evolve(B.product_state(N, sites), dt * steps)
        assert np.max(np.abs(psi[r * N ** 3:(r + 1) * N ** 3] - ref)) <= 1e-10


@pytest.mark.parametrize("acc", ["kahan", "plain"])
def test_three_walkers_c64(acc):
    """Complex64, 150 steps at tol 1e-7.  Against exact evolution the bar is
    the truncation budget (at most tol per step, 150 steps: 1.5e-5) plus
    rounding, held to 2e-5.  Against the oracle's Taylor map at the order
    the plan applies, only the FP32 rounding of the stored state is left: at
    most ~6e-8 per amplitude per step, accumulating as a random walk,
    sqrt(150) * 6e-8 = 7.3e-7 for amplitudes of size <= 1, held to 1e-6."""
    say(f"case: m=3 N=12 c64 {acc}, 150 steps")
    N, R, dt, steps = 12, 2, 0.02, 150
    reals = reals3(N, R, 2)
    sites = [4, 6, 7]
    plan = gpu_plan(m=3, statistics="distinguishable", boundary="open", interaction="nearest", dtype="c64",
                    accumulation=acc, reals=reals, dt=dt, tol=1e-7, sites=sites)
    plan.propagate(steps)
    psi = plan.state_numpy()
    worst = 0.0
    for r, (n, J, eps, U) in enumerate(reals):
        H = Hm.hamiltonian(N, 3, J, eps, U, B.DISTINGUISHABLE, "open", "nearest")
        ref = P.EDPropagator(H).evolve(B.product_state(N, sites), dt * steps)
        worst = max(worst, float(np.max(np.abs(psi[r * N ** 3:(r + 1) * N ** 3] - ref))))
    n2, _ = plan.realization_norms()
    say(f"  c64 {acc}: amplitude error {worst:.2e}, |norm - 1| {np.max(np.abs(np.sqrt(n2) - 1)):.1e}")
    assert worst <= 2e-5
    order = int(plan.orders().max())   # three-particle steps apply the batch's largest order
    map_err = 0.0
    for r, (n, J, eps, U) in enumerate(reals):
        H = Hm.hamiltonian(N, 3, J, eps, U, B.DISTINGUISHABLE, "open", "nearest")
        ref, _, _ = P.evolve_taylor(H, B.product_state(N, sites), dt, steps, order=order)
        map_err = max(map_err, float(np.max(np.abs(psi[r * N ** 3:(r + 1) * N ** 3] - ref))))
    say(f"  c64 {acc}: against the oracle's map at order {order}: {map_err:.2e}")
    assert map_err <= 1e-6


def test_full_lattice_window_against_oracle():
    """The three-walker workload's lattice (N = 256, nearest-neighbour U = 1,
    eps ~ U[-1, 1], start (127, 128, 129), dt = 0.02): after 5 steps of n
    terms each walker has moved at most 5 n nodes, so the full-lattice state
    equals the evolution on the window of nodes 96..159 (which contains every
    reachable node; the truncated map is the same on both) -- checked for 4
    realisations, with norm and occupation / pair sum rules on the whole
    lattice."""
    w = C5()
    R, steps, lo, hi = 4, 5, 96, 160
    say(f"case: {w.name} N={w.N} R={R} {steps} steps, window [{lo},{hi})")
    reals = w.all_realizations(range(R))
    plan = gpu_plan(m=3, statistics="distinguishable", boundary="open", interaction="nearest", dtype="c64",
                    reals=reals, dt=w.dt, tol=w.tol, observables=3, sites=list(w.start))
    n = int(plan.orders().max())
    assert w.start[0] - lo > steps * n and hi - 1 - w.start[2] >= steps * n
    out = plan.propagate(steps, steps, 3)
    psi = plan.state_numpy().reshape(R, w.N, w.N, w.N)
    M = hi - lo
    worst = 0.0
    for r, (N, J, eps, U) in enumerate(reals[:2]):
        Hw = Hm.hamiltonian(M, 3, J[lo:hi - 1], eps[lo:hi], U, B.DISTINGUISHABLE, "open", "nearest")
        ref, _, _ = P.evolve_taylor(Hw, B.product_state(M, [s - lo for s in w.start]), w.dt, steps, order=n)
        got = psi[r, lo:hi, lo:hi, lo:hi].reshape(-1)
        worst = max(worst, float(np.max(np.abs(got - ref))))
        rest = psi[r].copy()
        rest[lo:hi, lo:hi, lo:hi] = 0
        assert not rest.any()          # nothing outside the reachable window
    occ, pair = out[-1][:w.N], out[-1][w.N:].reshape(w.N, w.N)
    n2, _ = plan.realization_norms()
    say(f"  window amplitude error {worst:.2e}; sum occ {occ.sum():.7f}; |norm-1| {np.max(np.abs(np.sqrt(n2)-1)):.1e}")
    assert worst <= 1e-5
    assert abs(occ.sum() - 3) < 1e-5
    assert np.max(np.abs(pair.sum(axis=1) - 2 * occ)) < 1e-5
    assert np.max(np.abs(pair - pair.T)) < 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("K,order,boundary", [(3, 6, "open"), (3, 7, "open"), (2, 5, "periodic"), (1, 3, "open")])
def test_three_walkers_product_form(K, order, boundary, dtype):
    """Product form of the step (the order-n Taylor polynomial factored over
    its roots, at most K factors per pass, each pass reading and writing
    one state): one step on a 70-site chain (several tiles, every lane) of
    orders 3..7 against the oracle's Taylor map of the same order
    (complex128 1e-12; complex64 5e-9), and against the chained passes to
    rounding.  The truncation estimate is a bound on the last term, so it
    is at least the chained passes' exact one."""
    N, dt = 70 if boundary == "open" else 37, 0.02
    reals = reals3(N, 1, 7, boundary)
    say(f"case: m=3 product form N={N} {boundary} K={K} order={order} {dtype}")
    g = np.random.default_rng(12)
    D = N ** 3
    psi0 = g.standard_normal(D) + 1j * g.standard_normal(D)
    psi0 /= np.linalg.norm(psi0)

    def run(form):
        plan = gpu_plan(m=3, statistics="distinguishable", boundary=boundary, interaction="nearest", dtype=dtype,
                        reals=reals, dt=dt, order=order, launch={"terms_per_pass": K, "three_form": form})
        plan.set_state_numpy(psi0)
        plan.propagate(1)
        return plan.state_numpy(), plan.realization_norms()

    psi, (n2, t2) = run(1)
    psi_c, (n2_c, t2_c) = run(0)
    _, J, eps, U = reals[0]
    H = Hm.hamiltonian(N, 3, J, eps, U, B.DISTINGUISHABLE, boundary, "nearest")
    ref, _, _ = P.evolve_taylor(H, psi0, dt, 1, order=order)
    err = np.max(np.abs(psi - ref))
    d = np.max(np.abs(psi.astype(np.complex128) - psi_c.astype(np.complex128)))
    say(f"  max |psi - oracle map| = {err:.2e}, |product - chained| = {d:.2e}, "
        f"tail^2 product {t2[0]:.3e} chained {t2_c[0]:.3e}")
    bar = 1e-12 if dtype == "c128" else 5e-9
    assert err <= bar
    assert d <= 2 * bar
    assert abs(n2[0] - n2_c[0]) <= (1e-12 if dtype == "c128" else 1e-6)
    if order > K:
        assert t2[0] >= t2_c[0] * (1 - 1e-6)
    else:
        assert abs(t2[0] - t2_c[0]) <= 1e-6 * t2_c[0]
