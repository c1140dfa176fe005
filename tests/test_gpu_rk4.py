"""GPU parity of the Runge-Kutta propagator (Alg. 2): the library runs it as
the degree-4 Taylor step, one fused pass per step; the oracle runs the four
stages K1..K4 of Alg. 2 one matrix-vector product at a time.  They agree to
rounding, including the method's loss of norm (RK4 is not unitary)."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import propagate as P

from _helpers import gpu_plan, gpu_to_oracle, oracle_H, say

pytestmark = pytest.mark.gpu


def reals_for(Ns, seed):
    g = np.random.default_rng(seed)
    return [(N, 1 + 0.2 * g.standard_normal(N - 1), g.uniform(-0.5, 0.5, N), float(g.uniform(0.5, 2.0))) for N in Ns]


def rk4_plan(stat, dtype, acc, reals, dt, sites, P_=1):
    from paper_1612_00746_amd import Plan, make_problem
    from _helpers import pack
    Ns, J, eps, U = pack(reals)
    pr, keep = make_problem(2, len(Ns), Ns, dt, statistics=stat, dtype=dtype, accumulation=acc, method="rk4")
    plan = Plan(pr)
    plan._keep.append(keep)
    plan.set_launch(cols_per_lane=P_)
    plan.set_params(J, eps, U)
    plan.bind()
    plan.init_product_state(sites)
    return plan


@pytest.mark.parametrize("stat", ["distinguishable", "boson"])
def test_rk4_c128_matches_the_stagewise_oracle(stat):
    """c128, dt = 0.04, 150 steps: amplitudes within 1e-12 of the oracle's
    Alg. 2 stages, squared norms within 1e-12 of the oracle's (both drift
    from 1 by the method's own error)."""
    sb = B.BOSON if stat == "boson" else B.DISTINGUISHABLE
    reals = reals_for([40, 33, 70], 21)
    sites = [12, 13]
    dt, steps = 0.04, 150
    say(f"case: RK4 c128 {stat}, N={[r[0] for r in reals]}, dt={dt}, {steps} steps")
    plan = rk4_plan(stat, "c128", "plain", reals, dt, sites)
    assert list(plan.orders()) == [4] * len(reals)
    plan.propagate(steps)
    psi = plan.state_numpy()
    off = plan.layout()
    n2, _ = plan.realization_norms()
    for r, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, sb, "open", "onsite", J, eps, U)
        ref = P.evolve_rk4(H, B.product_state(N, sites, sb), dt, steps)
        got = gpu_to_oracle(psi[off[r]:off[r + 1]], N, 2, sb)
        err = float(np.max(np.abs(got - ref)))
        nref = float(np.vdot(ref, ref).real)
        say(f"  r={r} N={N}: max |psi - oracle RK4| = {err:.2e}, norm^2 {n2[r]:.15f} vs {nref:.15f}")
        assert err <= 1e-12
        assert abs(n2[r] - nref) <= 1e-12
        assert abs(nref - 1.0) > 1e-10   # the method's own norm loss is visible


@pytest.mark.parametrize("P_", [1, 2])
def test_rk4_c64_matches_the_stagewise_oracle(P_):
    """complex64 with the compensated sum, both lane layouts: within the
    complex64 bar of the oracle's Alg. 2 stages."""
    reals = reals_for([64, 48, 100], 22)
    sites = [20, 21]
    dt, steps = 0.04, 150
    say(f"case: RK4 c64 kahan P={P_}, dt={dt}, {steps} steps")
    plan = rk4_plan("distinguishable", "c64", "kahan", reals, dt, sites, P_)
    plan.propagate(steps)
    psi = plan.state_numpy()
    off = plan.layout()
    worst = 0.0
    for r, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", "onsite", J, eps, U)
        ref = P.evolve_rk4(H, B.product_state(N, sites, B.DISTINGUISHABLE), dt, steps)
        worst = max(worst, float(np.max(np.abs(psi[off[r]:off[r + 1]] - ref))))
    say(f"  max |psi - oracle RK4| = {worst:.2e}")
    assert worst <= 2e-6
