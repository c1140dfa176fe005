"""GPU parity of time-dependent (switching) hopping noise: the library
flips each bond's +-a term on the device at the start of every step and
rewrites the hopping tables; the oracle replays the same documented draws
and rebuilds H every step (oracle.telegraph)."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import telegraph as T

from _helpers import gpu_plan, gpu_to_oracle, oracle_H, say

pytestmark = pytest.mark.gpu


def reals_for(Ns, seed):
    g = np.random.default_rng(seed)
    return [(N, 1 + 0.1 * g.standard_normal(N - 1), g.uniform(-0.3, 0.3, N), float(g.uniform(0.5, 2.0))) for N in Ns]


@pytest.mark.parametrize("stat,launch", [("distinguishable", None), ("boson", None),
                                         ("distinguishable", {"use_graph": 1, "persistent": 1})])
def test_switching_noise_c128_against_the_oracle(stat, launch):
    """c128, order 10, dt = 0.05, 40 steps, a = 0.3, rate 4 (flip
    probability 0.18 per step): every realisation within 1e-12 of the
    oracle's step-by-step evolution, and far from the static-noise run."""
    sb = B.BOSON if stat == "boson" else B.DISTINGUISHABLE
    reals = reals_for([12, 15, 12], 41)
    sites = [4, 6]
    dt, steps, order, amp, rate, seed = 0.05, 40, 10, 0.3, 4.0, 99
    say(f"case: switching noise c128 {stat}, launch {launch}, N={[r[0] for r in reals]}")
    from paper_1612_00746_amd import Plan, make_problem
    from _helpers import pack
    Ns, J, eps, U = pack(reals)
    pr, keep = make_problem(2, len(Ns), Ns, dt, statistics=stat, dtype="c128", accumulation="plain",
                            taylor_order=order)
    plan = Plan(pr)
    plan._keep.append(keep)
    if launch:
        plan.set_launch(**launch)
    plan.set_params(J, eps, U)
    plan.set_telegraph(amp, rate, seed)
    plan.bind()
    plan.init_product_state(sites)
    plan.propagate(steps)
    psi = plan.state_numpy()
    off = plan.layout()
    static = gpu_plan(m=2, statistics=stat, boundary="open", interaction="onsite", dtype="c128",
                      accumulation="plain", reals=reals, dt=dt, order=order, sites=sites)
    static.propagate(steps)
    ps = static.state_numpy()
    for r, (N, Jb, e, u) in enumerate(reals):
        ref = T.evolve(lambda Jt: oracle_H(N, 2, sb, "open", "onsite", Jt, e, u), Jb,
                       B.product_state(N, sites, sb), dt, steps, order, amp, rate, seed, r)
        got = gpu_to_oracle(psi[off[r]:off[r + 1]], N, 2, sb)
        err = float(np.max(np.abs(got - ref)))
        diff = float(np.max(np.abs(psi[off[r]:off[r + 1]] - ps[off[r]:off[r + 1]])))
        say(f"  r={r} N={N}: max |psi - oracle| = {err:.2e}; vs static noise {diff:.2e}")
        assert err <= 1e-12
        assert diff > 1e-3
