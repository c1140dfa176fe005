"""GPU parity of per-realisation Taylor orders (Alg. 3 with an a-priori
order per realisation): a batch whose realisations need different orders
runs each one at its own order, grouped into one launch per order.  Checked
against the oracle's FP64 Taylor map at each realisation's order (computed
here from the documented bound, not taken from the library), across launch
forms, and through the truncation estimate, which must follow the order
that was applied.  Gradients apply the batch's largest order to every
realisation."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import propagate as P

from _helpers import gershgorin_x, gpu_plan, gpu_to_oracle, oracle_H, reference_order, say, tail_bound

pytestmark = pytest.mark.gpu

DT, TOL = 0.03, 1e-8


def mixed_reals(seed):
    """Realisations with hopping scales 0.7 to 1.8: orders 5 to 7, all
    within the fused pipeline's depth at one and two columns per lane."""
    g = np.random.default_rng(seed)
    out = []
    for N, s in ((40, 0.7), (70, 1.8), (33, 0.7), (64, 1.8), (129, 1.2)):
        out.append((N, s * (1 + 0.1 * g.standard_normal(N - 1)), g.uniform(-0.5, 0.5, N), float(g.uniform(0.5, 2.0))))
    return out


def expected_orders(reals, m=2):
    return [reference_order(J, eps, U, m, DT, TOL) for (_, J, eps, U) in reals]


def test_each_realisation_runs_its_own_order():
    """c128, 20 steps: every realisation equals the oracle's map at its own
    order to 1e-12, and differs from the map at the batch's largest order
    (so the check can tell the two apart)."""
    reals = mixed_reals(11)
    want = expected_orders(reals)
    say(f"case: per-realisation orders {want}, c128, N={[r[0] for r in reals]}, 20 steps")
    assert len(set(want)) >= 2
    sites = [10, 11]
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c128",
                    accumulation="plain", reals=reals, dt=DT, tol=TOL, sites=sites)
    assert list(plan.orders()) == want
    plan.propagate(20)
    psi = plan.state_numpy()
    off = plan.layout()
    nmax = max(want)
    for r, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", "onsite", J, eps, U)
        psi0 = B.product_state(N, sites, B.DISTINGUISHABLE)
        ref, _, _ = P.evolve_taylor(H, psi0, DT, 20, order=want[r])
        got = gpu_to_oracle(psi[off[r]:off[r + 1]], N, 2, B.DISTINGUISHABLE)
        err = float(np.max(np.abs(got - ref)))
        say(f"  r={r} N={N} order {want[r]}: max |psi - oracle| = {err:.2e}")
        assert err <= 1e-12
        if want[r] < nmax:
            alt, _, _ = P.evolve_taylor(H, psi0, DT, 20, order=nmax)
            assert float(np.max(np.abs(got - alt))) > 1e3 * max(err, 1e-15)


@pytest.mark.parametrize("dtype,acc", [("c64", "kahan"), ("c128", "plain")])
def test_per_order_launch_forms_are_bitwise_identical(dtype, acc):
    """Regular, persistent and graph-replayed per-order launches, at one and
    two columns per lane, give the same bits per launch shape family."""
    reals = mixed_reals(12)
    say(f"case: per-order launch forms, {dtype} {acc}, orders {expected_orders(reals)}")
    kw = dict(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype=dtype,
              accumulation=acc, reals=reals, dt=DT, tol=TOL, sites=[12, 13])
    for P_ in (1, 2):
        base = gpu_plan(**kw, launch={"cols_per_lane": P_})
        base.propagate(7)
        ref = base.state_numpy()
        for launch in ({"persistent": 1}, {"persistent": 1, "use_graph": 1}, {"use_graph": 1, "waves_per_block": 1}):
            p = gpu_plan(**kw, launch={"cols_per_lane": P_, **launch})
            p.propagate(7)
            assert np.array_equal(p.state_numpy(), ref), (P_, launch)


@pytest.mark.parametrize("acc", ["kahan", "plain"])
def test_two_order_launches_match_separate_launches(acc):
    """Complex64 at two columns per lane launches orders n and n - 1
    together (each item branching to its own pipeline); one column per lane
    launches each order alone.  The full-grid arithmetic is the same at one
    and two columns per lane, so the states agree bit for bit, and they
    differ from a run with every realisation at the largest order."""
    reals = mixed_reals(15)
    want = expected_orders(reals)
    say(f"case: two-order launch vs separate launches, c64 {acc}, orders {want}")
    assert len(set(want)) >= 2
    kw = dict(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
              accumulation=acc, reals=reals, dt=DT, sites=[14, 15])
    out = {}
    for P_ in (1, 2):
        plan = gpu_plan(**kw, tol=TOL, launch={"cols_per_lane": P_, "persistent": 1})
        plan.propagate(11)
        out[P_] = plan.state_numpy()
    assert np.array_equal(out[1], out[2])
    fixed = gpu_plan(**kw, tol=0.0, order=max(want), launch={"cols_per_lane": 2})
    fixed.propagate(11)
    assert not np.array_equal(fixed.state_numpy(), out[2])


@pytest.mark.parametrize("dtype,bar", [("c128", 1e-9), ("c64", 1e-4)])
def test_truncation_estimate_follows_the_applied_order(dtype, bar):
    """After four steps the squared truncation estimate of realisation r is
    ||Phi^(n_r)||^2 f(x_r, n_r)^2, with Phi^(n) = (-i dt H)^n psi / n! of the
    state the last step started from, f the remainder factor of the documented
    bound and n_r the realisation's own order.  complex128 sums ||Phi^(n)||^2
    in FP64 (relative bar 1e-9); complex64 sums it per column in FP32 and
    widens the column sums to FP64 (it only scales the bound): relative bar
    1e-4, which covers the FP32 state and the FP32 column sums (one rounding
    of 6e-8 per row, at most 1024 rows)."""
    reals = mixed_reals(13)
    want = expected_orders(reals)
    say(f"case: truncation estimate {dtype}, orders {want}")
    sites = [5, 9]
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype=dtype,
                    accumulation="plain" if dtype == "c128" else "kahan", reals=reals, dt=DT, tol=TOL, sites=sites)
    plan.propagate(4)
    _, t2 = plan.realization_norms()
    for r, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", "onsite", J, eps, U)
        # the oracle's state after three steps at this realisation's order
        term, _, _ = P.evolve_taylor(H, B.product_state(N, sites, B.DISTINGUISHABLE), DT, 3, order=want[r])
        for j in range(1, want[r] + 1):
            term = (-1j * DT / j) * (H @ term)
        x = gershgorin_x(J, eps, U, 2, DT)
        ref = float(np.vdot(term, term).real) * tail_bound(x, want[r]) ** 2
        say(f"  r={r} order {want[r]}: tail2 {t2[r]:.6e} vs {ref:.6e} (relative {abs(t2[r] - ref) / ref:.1e})")
        assert abs(t2[r] - ref) <= bar * ref


def test_gradient_runs_one_order_for_the_batch():
    """The adjoint inverts one polynomial: with realisations of different
    orders the gradient's forward pass applies the largest to all, so its
    loss equals the loss after propagating a plan fixed at that order."""
    N, dt, steps = 14, DT, 12
    g = np.random.default_rng(14)
    reals = [(N, s * (1 + 0.1 * g.standard_normal(N - 1)), g.uniform(-0.3, 0.3, N), 1.0) for s in (0.7, 1.8, 0.7)]
    want = expected_orders(reals)
    say(f"case: gradient with orders {want}, c128 bosons N={N}")
    assert len(set(want)) >= 2
    sw = (np.arange(N) >= 9).astype(float)
    kw = dict(m=2, statistics="boson", boundary="open", interaction="onsite", dtype="c128", accumulation="plain",
              reals=reals, dt=dt, sites=[3, 4])
    mixed = gpu_plan(**kw, tol=TOL)
    loss, gJ, gE = mixed.gradient(steps, 4, sw, "product")
    fixed = gpu_plan(**kw, order=max(want), tol=0.0)
    fixed.propagate(steps)
    ref = fixed.loss(sw, "product")
    say(f"  gradient loss {loss:.15f}, fixed-order loss {ref:.15f}")
    assert abs(loss - ref) <= 1e-14
    assert np.all(np.isfinite(gJ)) and np.all(np.isfinite(gE))


@pytest.mark.parametrize("dtype,P_", [("c128", 1), ("c128", 2), ("c64", 1), ("c64", 2)])
@pytest.mark.parametrize("order", [1, 2, 3])
def test_lowest_orders_against_the_oracle_map(dtype, P_, order):
    """The shallowest pipelines (one to three terms; the unrolled block is
    then three rows) on a ragged batch — chains of 2, 3, 65 and 130 sites,
    one to three bands — against the oracle's Taylor map of the same order."""
    g = np.random.default_rng(50 + order)
    reals = [(N, 1 + 0.1 * g.standard_normal(N - 1), g.uniform(-0.3, 0.3, N), float(g.uniform(0.5, 2.0)))
             for N in (2, 3, 65, 130)]
    sites = [0, 1]
    dt, steps = 0.01, 15
    say(f"case: order {order}, {dtype}, P={P_}, N={[r[0] for r in reals]}")
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype=dtype,
                    accumulation="kahan" if dtype == "c64" else "plain", reals=reals, dt=dt, order=order,
                    launch={"cols_per_lane": P_}, sites=sites)
    plan.propagate(steps)
    psi = plan.state_numpy()
    off = plan.layout()
    worst = 0.0
    for r, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", "onsite", J, eps, U)
        ref, _, _ = P.evolve_taylor(H, B.product_state(N, sites, B.DISTINGUISHABLE), dt, steps, order=order)
        worst = max(worst, float(np.max(np.abs(psi[off[r]:off[r + 1]] - ref))))
    say(f"  max |psi - oracle map| = {worst:.2e}")
    assert worst <= (1e-13 if dtype == "c128" else 1e-6)
