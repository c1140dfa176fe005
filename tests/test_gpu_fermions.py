"""GPU parity of two fermions on the chain stencil (Sec. 1-2: walks depend
on the particles' statistics).  The library stores the antisymmetric
function phi(x1, x2) on the triangle x1 <= x2 with its diagonal held at 0;
the oracle evolves the coefficients in the normalised antisymmetric basis
(pairs x1 < x2, H_A = A^T H A).  Complex128 parity against exact
diagonalisation (1e-10), complex64 against the same within the complex64
bar, observables, layouts, launch shapes and the refusals (two fermions
on one node, rings, gradients)."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import observables as O
from oracle import propagate as P

from _helpers import gpu_plan, gpu_to_oracle, gpu_tri_diagonal, oracle_H, say

pytestmark = pytest.mark.gpu


def reals_for(N, R, seed):
    g = np.random.default_rng(seed)
    return [(N, 1 + 0.2 * g.standard_normal(N - 1), g.uniform(-0.5, 0.5, N), float(g.uniform(0.5, 2.0)))
            for _ in range(R)]


@pytest.mark.parametrize("N,interaction,sites,launch", [
    (14, "nearest", [5, 8], None),
    (14, "onsite", [9, 4], None),
    (71, "nearest", [30, 41], None),
    (71, "nearest", [40, 31], {"cols_per_lane": 2}),
    (40, "nearest", [19, 20], {"chunked": 1}),
])
def test_two_fermions_c128_against_ed(N, interaction, sites, launch):
    R, dt, steps = 3, 0.05, 60
    reals = reals_for(N, R, 3)
    say(f"case: fermions N={N} {interaction} start {sites} launch {launch} c128, {steps} steps")
    plan = gpu_plan(m=2, statistics="fermion", boundary="open", interaction=interaction, dtype="c128",
                    reals=reals, dt=dt, tol=1e-14, observables=3, sites=sites, launch=launch)
    out = plan.propagate(steps, steps, 3)
    psi = plan.state_numpy()
    off = plan.layout()
    st = B.basis_states(N, 2, B.FERMION)
    worst, occ, pair, diag = 0.0, [], [], 0.0
    for r, (n, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, B.FERMION, "open", interaction, J, eps, U)
        ref = P.EDPropagator(H).evolve(B.product_state(N, sites, B.FERMION), dt * steps)
        got = psi[off[r]:off[r + 1]]
        worst = max(worst, float(np.max(np.abs(gpu_to_oracle(got, N, 2, B.FERMION) - ref))))
        diag = max(diag, float(np.max(np.abs(gpu_tri_diagonal(got, N)))))
        occ.append(O.occupation(ref, st, N))
        pair.append(O.pair_correlation(ref, st, N))
    e_occ = float(np.max(np.abs(out[-1][:N] - O.ensemble_mean(occ))))
    e_pair = float(np.max(np.abs(out[-1][N:].reshape(N, N) - O.ensemble_mean(pair))))
    n2, _ = plan.realization_norms()
    say(f"  amplitude {worst:.2e}, occupation {e_occ:.2e}, pair {e_pair:.2e}, diagonal {diag:.1e}, "
        f"|norm^2 - 1| {np.max(np.abs(n2 - 1)):.1e}")
    assert worst <= 1e-10 and e_occ <= 1e-10 and e_pair <= 1e-10
    assert diag == 0.0                         # Pauli: no two fermions on one node, ever
    assert np.max(np.abs(n2 - 1)) < 1e-12
    assert np.max(np.abs(np.diag(out[-1][N:].reshape(N, N)))) == 0.0


def test_two_fermions_c64():
    N, R, dt, steps = 48, 4, 0.05, 200
    reals = reals_for(N, R, 4)
    sites = [20, 27]
    say(f"case: fermions N={N} c64, {steps} steps")
    plan = gpu_plan(m=2, statistics="fermion", boundary="open", interaction="nearest", dtype="c64", reals=reals,
                    dt=dt, tol=1e-7, sites=sites)
    plan.propagate(steps)
    psi = plan.state_numpy()
    off = plan.layout()
    worst = 0.0
    for r, (n, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, B.FERMION, "open", "nearest", J, eps, U)
        ref = P.EDPropagator(H).evolve(B.product_state(N, sites, B.FERMION), dt * steps)
        worst = max(worst, float(np.max(np.abs(gpu_to_oracle(psi[off[r]:off[r + 1]], N, 2, B.FERMION) - ref))))
    n2, _ = plan.realization_norms()
    say(f"  amplitude {worst:.2e}, |norm - 1| {np.max(np.abs(np.sqrt(n2) - 1)):.1e}")
    assert worst <= 1e-6
    assert np.max(np.abs(np.sqrt(n2) - 1)) <= 1e-6


def test_fermion_refusals():
    """Two fermions on one start node, a ring, and gradients are refused
    with clear errors."""
    from paper_1612_00746_amd import CtqwError, Plan, make_problem
    reals = reals_for(10, 2, 5)
    plan = gpu_plan(m=2, statistics="fermion", boundary="open", interaction="nearest", dtype="c128", reals=reals,
                    dt=0.05, tol=1e-12)
    with pytest.raises(CtqwError) as e:
        plan.init_product_state([3, 3])
    assert e.value.status == 1
    pr, _ = make_problem(2, 2, 10, 0.05, statistics="fermion", boundary="periodic", taylor_tol=1e-12)
    with pytest.raises(CtqwError) as e:
        Plan(pr)
    assert e.value.status == 2
    plan.init_product_state([3, 6])
    with pytest.raises(CtqwError) as e:
        plan.gradient(4, 2, np.ones(10))
    assert e.value.status == 2
