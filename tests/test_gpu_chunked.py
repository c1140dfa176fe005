"""GPU parity of chunked steps: Taylor orders above the fused pipeline's
depth run as passes of K terms (8 complex64, 4 complex128) that carry the
partial sum and the last term between passes.  Checked against the
oracle's FP64 Taylor map of the same order, against the fused kernel at an
order both can run, across launch forms, and through the adjoint's
recomputation."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import propagate as P

from _helpers import gpu_plan, gpu_to_oracle, oracle_H, say

pytestmark = pytest.mark.gpu


def reals2(Ns, seed):
    g = np.random.default_rng(seed)
    return [(N, 1 + 0.1 * g.standard_normal(N - 1), g.uniform(-0.5, 0.5, N), float(g.uniform(0.5, 2.0)))
            for N in Ns]


def max_err_vs_taylor(plan, reals, stat, sites, dt, steps, order):
    psi = plan.state_numpy()
    off = plan.layout()
    sb = B.BOSON if stat == "boson" else B.DISTINGUISHABLE
    worst = 0.0
    for r, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, sb, "open", "onsite", J, eps, U)
        ref, _, _ = P.evolve_taylor(H, B.product_state(N, sites, sb), dt, steps, order=order)
        got = gpu_to_oracle(psi[off[r]:off[r + 1]], N, 2, sb)
        worst = max(worst, float(np.max(np.abs(got - ref))))
    return worst


@pytest.mark.parametrize("stat", ["distinguishable", "boson"])
def test_order_20_c128_matches_the_oracle_taylor_map(stat):
    """Order 20 at dt = 0.3 (5 passes of 4 terms, 130 columns = 3 bands):
    the state after 25 steps equals the oracle's order-20 map to 1e-11."""
    say(f"case: chunked c128 {stat}, order 20, N=[130, 47], 25 steps")
    reals = reals2([130, 47], 3)
    sites = [20, 21]
    plan = gpu_plan(m=2, statistics=stat, boundary="open", interaction="onsite", dtype="c128", reals=reals,
                    dt=0.3, order=20, tol=0.0, sites=sites)
    plan.propagate(25)
    err = max_err_vs_taylor(plan, reals, stat, sites, 0.3, 25, 20)
    n2, t2 = plan.realization_norms()
    say(f"  max |psi - oracle| = {err:.2e}, |norm - 1| = {np.max(np.abs(np.sqrt(n2) - 1)):.1e}")
    assert err <= 1e-11
    assert np.max(np.abs(np.sqrt(n2) - 1)) < 1e-8


@pytest.mark.parametrize("dtype,acc,bar", [("c128", "plain", 1e-13), ("c64", "kahan", 2e-6)])
def test_forced_passes_match_the_fused_kernel(dtype, acc, bar):
    """Order 7: the chunked passes (forced) and the fused pipeline evaluate
    the same polynomial; they differ only by the rounding of the partial sum
    stored between passes."""
    say(f"case: chunked vs fused, {dtype} {acc}, order 7, 60 steps")
    reals = reals2([100, 64, 33], 4)
    kw = dict(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype=dtype,
              accumulation=acc, reals=reals, dt=0.05, order=7, tol=0.0, sites=[16, 17])
    fused = gpu_plan(**kw)
    chunked = gpu_plan(**kw, launch={"chunked": 1})
    fused.propagate(60)
    chunked.propagate(60)
    d = float(np.max(np.abs(fused.state_numpy().astype(np.complex128) - chunked.state_numpy())))
    say(f"  max |fused - chunked| = {d:.2e}")
    assert d <= bar
    err = max_err_vs_taylor(chunked, reals, "distinguishable", [16, 17], 0.05, 60, 7)
    say(f"  chunked vs oracle map: {err:.2e}")
    # complex64: FP32 rounding of the stored state, at most ~6e-8 per
    # amplitude per step, as a random walk over 60 steps: 4.6e-7.
    assert err <= (1e-12 if dtype == "c128" else 5e-7)


def test_chunked_launch_forms_are_bitwise_identical():
    """Regular, persistent and graph-replayed chunked steps give the same
    bits (each item's arithmetic does not depend on which wave runs it), and
    the complex64 passes follow the oracle's FP64 map of the same order."""
    say("case: chunked launch forms, c64 order 17")
    reals = reals2([150, 90, 64], 5)
    kw = dict(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
              reals=reals, dt=0.2, order=17, tol=0.0, sites=[30, 31])
    ref = gpu_plan(**kw)
    ref.propagate(9)
    base = ref.state_numpy()
    for launch in ({"persistent": 1}, {"persistent": 1, "use_graph": 1}, {"waves_per_block": 1}):
        p = gpu_plan(**kw, launch=launch)
        p.propagate(9)
        assert np.array_equal(p.state_numpy(), base), launch
    # three passes of 8 terms in complex64 against the FP64 map of order 17
    err = max_err_vs_taylor(ref, reals, "distinguishable", [30, 31], 0.2, 9, 17)
    say(f"  c64 order 17 (3 passes) vs oracle map: {err:.2e}")
    assert err <= 2e-6


def test_adjoint_with_chunked_recomputation():
    """The adjoint recomputes checkpoint segments with the step kernels:
    with forced passes the gradient equals the fused one (c128, order 9)."""
    say("case: adjoint with chunked recomputation, c128 bosons N=12, order 9")
    N, R, dt, steps = 12, 2, 0.1, 24
    g = np.random.default_rng(6)
    reals = [(N, 1 + 0.1 * g.standard_normal(N - 1), g.uniform(-0.3, 0.3, N), 1.0) for _ in range(R)]
    sw = (np.arange(N) >= 8).astype(float)
    out = []
    for launch in (None, {"chunked": 1}):
        plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype="c128",
                        reals=reals, dt=dt, order=9, tol=0.0, sites=[3, 4], launch=launch)
        out.append(plan.gradient(steps, 5, sw, "product"))
    (l0, gJ0, gE0), (l1, gJ1, gE1) = out
    say(f"  loss {l0:.14f} / {l1:.14f}; max grad diff {max(np.max(np.abs(gJ0 - gJ1)), np.max(np.abs(gE0 - gE1))):.1e}")
    assert abs(l0 - l1) < 1e-13
    assert np.allclose(gJ0, gJ1, rtol=0, atol=1e-12) and np.allclose(gE0, gE1, rtol=0, atol=1e-12)
