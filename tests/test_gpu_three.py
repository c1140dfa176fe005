"""GPU parity for three distinguishable walkers (one Taylor term per pass):
against the oracle's exact evolution on small lattices, and on the full
N = 256 lattice against the oracle on the window the walkers can reach."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import hamiltonian as Hm
from oracle import observables as O
from oracle import propagate as P
from workloads import C5

from _helpers import gpu_plan, say

pytestmark = pytest.mark.gpu


def reals3(N, R, seed, boundary="open"):
    g = np.random.default_rng(seed)
    nb = N if boundary == "periodic" else N - 1
    return [(N, 1 + 0.2 * g.standard_normal(nb), g.uniform(-1, 1, N), float(g.uniform(0.5, 1.5))) for _ in range(R)]


@pytest.mark.parametrize("N,boundary,interaction", [(7, "open", "nearest"), (10, "open", "nearest"),
                                                    (6, "periodic", "onsite"), (5, "periodic", "nearest")])
def test_three_walkers_c128_against_ed(N, boundary, interaction):
    say(f"case: m=3 N={N} {boundary} {interaction} c128, 40 steps")
    R, dt, steps = 3, 0.02, 40
    reals = reals3(N, R, 1, boundary)
    sites = [1, N // 2, N - 2]
    plan = gpu_plan(m=3, statistics="distinguishable", boundary=boundary, interaction=interaction, dtype="c128",
                    reals=reals, dt=dt, tol=1e-14, observables=3, sites=sites)
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
    say(f"  amplitude {worst:.2e}, occupation {e_occ:.2e}, pair {e_pair:.2e}")
    assert worst <= 1e-10 and e_occ <= 1e-10 and e_pair <= 1e-10
    assert abs(out[0][:N].sum() - 3) < 1e-12


@pytest.mark.parametrize("acc", ["kahan", "plain"])
def test_three_walkers_c64(acc):
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
