"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
identical seeded inputs, element by element.

Bars: complex128 state <= 1e-10 max-abs amplitude and occupation error
(the target set for the FP64 path); complex64 bars are stated per test and
derived from the single-precision rounding of the stored state (about
6e-8 relative per step, growing like the square root of the step count)."""

import math

import numpy as np
import pytest

from oracle import basis as B
from oracle import observables as O
from oracle import propagate as P
from workloads import C1, Noise, Workload, scaled

from _helpers import gpu_plan, gpu_to_oracle, oracle_H, oracle_to_gpu, say

pytestmark = pytest.mark.gpu

C128_BAR = 1e-10


def ed_states(reals, m, statistics, boundary, interaction, sites, times):
    out = []
    for k, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, m, statistics, boundary, interaction, J, eps, U)
        s = sites[k] if np.ndim(sites) == 2 else sites
        out.append(P.EDPropagator(H).evolve_many(B.product_state(N, list(s), statistics), times))
    return out


ED_MAX_DIM = 3000


def oracle_final(N, J, eps, U, m, statistics, boundary, interaction, s, t, dt):
    """Exact evolution to time t: ED for small dimensions, the oracle's
    Taylor route with tolerance 1e-15 per step (pinned against ED) above."""
    H = oracle_H(N, m, statistics, boundary, interaction, J, eps, U)
    psi0 = B.product_state(N, list(s), statistics)
    if H.shape[0] <= ED_MAX_DIM:
        return P.EDPropagator(H).evolve(psi0, t)
    steps = int(round(t / dt))
    psi, _, _ = P.evolve_taylor(H, psi0, dt, steps, tol=1e-15)
    return psi


def compare_final(plan, reals, m, statistics, boundary, interaction, sites, t, bar, dt=0.05):
    psi = plan.state_numpy()
    off = plan.layout()
    worst = 0.0
    for k, (N, J, eps, U) in enumerate(reals):
        s = sites[k] if np.ndim(sites) == 2 else sites
        ref = oracle_final(N, J, eps, U, m, statistics, boundary, interaction, s, t, dt)
        got = gpu_to_oracle(psi[off[k]:off[k + 1]], N, m, statistics)
        worst = max(worst, float(np.max(np.abs(got - ref))))
    say(f"  max |psi_gpu - psi_ed| = {worst:.3e} (bar {bar:.1e})")
    assert worst <= bar
    return worst


def random_reals(Ns, boundary="open", seed=0, U=(0.0, 2.0), eps=0.5, Jsig=0.2):
    g = np.random.default_rng(seed)
    out = []
    for N in Ns:
        nb = N if boundary == "periodic" else N - 1
        out.append((N, 1 + Jsig * g.standard_normal(nb), g.uniform(-eps, eps, N), float(g.uniform(*U))))
    return out


# ------------------------------------------------------------ closed forms

def test_bessel_single_walker_c128():
    """One walker, uniform open chain N=256 from node 128, t = 10:
    psi_{128+n} = (-i)^n J_n(2t) (closed form)."""
    import scipy.special as ss
    say("case: m=1 N=256 c128 Bessel, dt=0.05, 200 steps")
    N, s, dt, steps = 256, 128, 0.05, 200
    reals = [(N, np.ones(N - 1), np.zeros(N), 0.0)]
    plan = gpu_plan(m=1, statistics="distinguishable", boundary="open", interaction="onsite",
                    dtype="c128", reals=reals, dt=dt, tol=1e-14, sites=[s])
    plan.propagate(steps)
    psi = plan.state_numpy()
    n = np.abs(np.arange(N) - s)
    expect = (-1j) ** n * ss.jv(n, 2 * dt * steps)
    err = np.max(np.abs(psi - expect))
    say(f"  max err vs Bessel = {err:.3e}")
    assert err <= C128_BAR


def test_config1_full_c128():
    """2 distinguishable walkers, N=16 open, J_i = 1 + U[-0.1, 0.1], 8
    realisations, start (7, 8), dt = 0.01 to t = 5, occupation every 0.1."""
    w = C1()
    say(f"case: {w.name} R={w.R} steps={w.n_steps}")
    reals = w.all_realizations()
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite",
                    dtype="c128", reals=reals, dt=w.dt, tol=w.tol, sites=list(w.start))
    occ = plan.propagate(w.n_steps, w.output_every, 1)
    assert occ.shape == (w.n_steps // w.output_every + 1, 16)
    times = np.arange(occ.shape[0]) * w.output_every * w.dt
    states = B.basis_states(16, 2)
    ref = ed_states(reals, 2, B.DISTINGUISHABLE, "open", "onsite", w.start, times)
    ens = np.array([O.ensemble_mean([O.occupation(ref[r][k], states, 16) for r in range(w.R)])
                    for k in range(len(times))])
    err = np.max(np.abs(occ - ens))
    say(f"  max occupation error over {len(times)} snapshots = {err:.3e}")
    assert err <= C128_BAR
    assert np.max(np.abs(occ.sum(axis=1) - 2.0)) < 1e-12
    compare_final(plan, reals, 2, B.DISTINGUISHABLE, "open", "onsite", w.start, w.n_steps * w.dt, C128_BAR)
    st = plan.stats()
    assert st.steps_done == w.n_steps and abs(st.max_norm - 1) < 1e-12 and st.flags == 0


# ------------------------------------------------------------- two particles

@pytest.mark.parametrize("P_", [1, 2])
def test_distinguishable_multiband_c128(P_):
    """Multi-band realisations.  Two columns per lane are compiled for FP64
    up to order 8, so that case runs a fixed order 8 against the oracle's
    fixed-order Taylor map."""
    say(f"case: m=2 dist open N=[100,150,64,65] c128 P={P_}")
    reals = random_reals([100, 150, 64, 65], seed=1)
    if P_ == 1:
        plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite",
                        dtype="c128", reals=reals, dt=0.05, tol=1e-14, launch={"cols_per_lane": P_},
                        sites=[40, 50])
        plan.propagate(60)
        compare_final(plan, reals, 2, B.DISTINGUISHABLE, "open", "onsite", [40, 50], 3.0, C128_BAR)
        return
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c128",
                    reals=reals, dt=0.02, order=8, tol=0.0, launch={"cols_per_lane": P_}, sites=[40, 50])
    plan.propagate(40)
    psi = plan.state_numpy()
    off = plan.layout()
    worst = 0.0
    for k, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", "onsite", J, eps, U)
        ref, _, _ = P.evolve_taylor(H, B.product_state(N, [40, 50]), 0.02, 40, order=8)
        worst = max(worst, float(np.max(np.abs(psi[off[k]:off[k + 1]] - ref))))
    say(f"  fixed order 8, 40 steps: max err vs oracle Taylor map {worst:.3e}")
    assert worst <= C128_BAR


@pytest.mark.parametrize("N", [2, 3, 70, 130])
def test_bosons_c128(N):
    say(f"case: m=2 bosons open N={N} c128")
    reals = random_reals([N, N], seed=2)
    s = [0, 1] if N <= 3 else [N // 2 - 1, N // 2]
    plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype="c128",
                    reals=reals, dt=0.05, tol=1e-14, sites=s)
    plan.propagate(40)
    compare_final(plan, reals, 2, B.BOSON, "open", "onsite", s, 2.0, C128_BAR)


def test_bosons_double_occupied_start_and_nearest():
    say("case: m=2 bosons N=40 start (20,20), nearest-neighbour U")
    reals = random_reals([40], seed=3)
    plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="nearest", dtype="c128",
                    reals=reals, dt=0.05, tol=1e-14, sites=[20, 20])
    plan.propagate(30)
    compare_final(plan, reals, 2, B.BOSON, "open", "nearest", [20, 20], 1.5, C128_BAR)


@pytest.mark.parametrize("interaction", ["onsite", "nearest"])
def test_periodic_c128(interaction):
    say(f"case: m=2 dist periodic N=[7,40,90] {interaction} c128")
    reals = random_reals([7, 40, 90], boundary="periodic", seed=4)
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="periodic", interaction=interaction,
                    dtype="c128", reals=reals, dt=0.05, tol=1e-14, sites=[1, 5])
    plan.propagate(40)
    compare_final(plan, reals, 2, B.DISTINGUISHABLE, "periodic", interaction, [1, 5], 2.0, C128_BAR)


def test_single_walker_periodic_and_uneven():
    say("case: m=1 periodic N=[3, 50, 300] c128")
    reals = random_reals([3, 50, 300], boundary="periodic", seed=5)
    plan = gpu_plan(m=1, statistics="distinguishable", boundary="periodic", interaction="onsite",
                    dtype="c128", reals=reals, dt=0.05, tol=1e-14, sites=[1])
    plan.propagate(50)
    compare_final(plan, reals, 1, B.DISTINGUISHABLE, "periodic", "onsite", [1], 2.5, C128_BAR)


def test_uneven_batch_c128_with_groups():
    Ns = [16, 33, 64, 100, 130, 16, 33]
    say(f"case: uneven batch N={Ns} c128, per-realisation start sites")
    reals = random_reals(Ns, seed=6, U=(0, 4))
    sites = np.array([[n // 2 - 1, n // 2] for n in Ns], dtype=np.int32)
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite",
                    dtype="c128", reals=reals, dt=0.05, tol=1e-14, sites=sites)
    occ = plan.propagate(40, 20, 1)
    assert list(plan.groups()) == [16, 33, 64, 100, 130]
    compare_final(plan, reals, 2, B.DISTINGUISHABLE, "open", "onsite", sites, 2.0, C128_BAR)
    # ensemble occupation of the N=16 group (realisations 0 and 5) at t=2
    ref = ed_states([reals[0], reals[5]], 2, B.DISTINGUISHABLE, "open", "onsite", sites[[0, 5]], [2.0])
    st = B.basis_states(16, 2)
    ens = O.ensemble_mean([O.occupation(ref[k][0], st, 16) for k in range(2)])
    assert np.max(np.abs(occ[-1][:16] - ens)) <= C128_BAR


def test_pair_correlation_c128():
    say("case: pair correlation m=2 dist N=24 and bosons N=24")
    for stat in ("distinguishable", "boson"):
        reals = random_reals([24, 24, 24], seed=7)
        plan = gpu_plan(m=2, statistics=stat, boundary="open", interaction="onsite", dtype="c128",
                        reals=reals, dt=0.05, tol=1e-14, observables=3, sites=[10, 13])
        out = plan.propagate(30, 30, 3)
        sb = B.BOSON if stat == "boson" else B.DISTINGUISHABLE
        ref = ed_states(reals, 2, sb, "open", "onsite", [10, 13], [1.5])
        st = B.basis_states(24, 2, sb)
        occ = O.ensemble_mean([O.occupation(ref[k][0], st, 24) for k in range(3)])
        G = O.ensemble_mean([O.pair_correlation(ref[k][0], st, 24) for k in range(3)])
        got_occ, got_G = out[-1][:24], out[-1][24:].reshape(24, 24)
        say(f"  {stat}: occ err {np.max(np.abs(got_occ - occ)):.2e} pair err {np.max(np.abs(got_G - G)):.2e}")
        assert np.max(np.abs(got_occ - occ)) <= C128_BAR
        assert np.max(np.abs(got_G - G)) <= C128_BAR


# ------------------------------------------------------------ zero on-site energies

@pytest.mark.parametrize("interaction", ["onsite", "nearest"])
@pytest.mark.parametrize("P_", [1, 2])
def test_zero_onsite_energies_c128(P_, interaction):
    """Without on-site energies the diagonal of H is the interaction alone
    and the step kernel skips the diagonal product on rows whose band has no
    interacting column.  Chains of several bands with eps = 0 and U != 0
    against the oracle's Taylor map of the same order (1e-12)."""
    say(f"case: eps = 0, m=2 dist open N=[150,300,200] c128 P={P_} {interaction}")
    reals = [(N, J, np.zeros(N), U) for (N, J, _, U) in random_reals([150, 300, 200], seed=3, U=(1.0, 3.0))]
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction=interaction, dtype="c128",
                    reals=reals, dt=0.05, order=8, tol=0.0, launch={"cols_per_lane": P_}, sites=[70, 75])
    plan.propagate(30)
    psi = plan.state_numpy()
    off = plan.layout()
    worst = 0.0
    for k, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", interaction, J, eps, U)
        ref, _, _ = P.evolve_taylor(H, B.product_state(N, [70, 75]), 0.05, 30, order=8)
        worst = max(worst, float(np.max(np.abs(psi[off[k]:off[k + 1]] - ref))))
    say(f"  max err vs oracle Taylor map {worst:.3e}")
    assert worst <= 1e-12


@pytest.mark.parametrize("P_", [1, 2])
def test_zero_onsite_energies_bitwise_c64(P_):
    """complex64: the diagonal-free rows give the same bits as the full
    stencil.  A batch with eps = 0 against the same batch with one on-site
    energy of 1e-300, which makes the kernel keep the diagonal product on
    every row but rounds to 0 in the FP32 tables."""
    say(f"case: eps = 0 vs eps with a 1e-300 entry, c64 P={P_}")
    base = [(N, J, np.zeros(N), U) for (N, J, _, U) in random_reals([150, 300, 64, 520], seed=4, U=(1.0, 3.0))]
    tiny = [(N, J, np.where(np.arange(N) == N - 1, 1e-300, 0.0), U) for (N, J, _, U) in base]
    out = []
    for reals in (base, tiny):
        plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
                        reals=reals, dt=0.05, tol=1e-7, launch={"cols_per_lane": P_}, sites=[30, 31])
        plan.propagate(25)
        out.append(plan.state_numpy())
    assert np.array_equal(out[0], out[1])


# ------------------------------------------------------------ launch shapes

def test_graph_replays_match_eager_launches():
    """The step loop captured in a HIP graph (with the persistent kernel and
    its per-wave item lists) and replayed several times, with eager work and
    synchronisation in between, gives the eager result after every replay."""
    say("case: hipGraph step loop vs eager, 4 replays of 6 steps")
    reals = random_reals([100, 33, 64], seed=14)
    eager = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
                     reals=reals, dt=0.05, tol=1e-7, launch={"persistent": 1}, sites=[20, 21])
    graph = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
                     reals=reals, dt=0.05, tol=1e-7, launch={"persistent": 1, "use_graph": 1}, sites=[20, 21])
    for rep in range(4):
        eager.propagate(6)
        graph.propagate(6)
        occ_g = graph.observe(1)
        occ_e = eager.observe(1)
        assert np.array_equal(graph.state_numpy(), eager.state_numpy()), f"replay {rep}"
        assert np.array_equal(occ_g, occ_e)
    # odd-length segments alternate the starting buffer
    eager.propagate(7, 7, 1)
    graph.propagate(7, 7, 1)
    assert np.array_equal(graph.state_numpy(), eager.state_numpy())
    assert graph.stats().steps_done == eager.stats().steps_done == 31


def test_timed_graph_replays_count_every_step_kernel():
    """Timing of captured step loops: each replay is bracketed by an event
    pair that counts for its steps, so the timed steps equal the steps taken,
    and a timed loop gives the untimed loop's state bit for bit (300 steps =
    graphs of 256 and 44 steps)."""
    say("case: timed hipGraph step loops, 2 x 300 steps")
    reals = random_reals([100, 33, 64], seed=16)
    kw = dict(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
              reals=reals, dt=0.05, tol=1e-7, launch={"persistent": 1, "use_graph": 1}, sites=[20, 21])
    plain, timed = gpu_plan(**kw), gpu_plan(**kw)
    timed.set_timing(True)
    for rep in (1, 2):
        plain.propagate(300)
        timed.propagate(300)
        ms, launches = timed.get_timing()
        say(f"  after {300 * rep} steps: {launches} timed launches, {ms:.3f} ms")
        assert launches == 300 * rep and ms > 0
        assert np.array_equal(plain.state_numpy(), timed.state_numpy())


def test_autotune_applies_and_caches_a_shape(tmp_path):
    """The autotuner picks a launch shape, writes it to the cache, a second
    plan of the same shape reads it back, and results do not depend on it."""
    say("case: autotune + cache on an uneven batch")
    reals = random_reals([64, 200, 130], seed=15)
    cache = str(tmp_path / "tune.jsonl")
    p1 = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
                  reals=reals, dt=0.05, tol=1e-7)
    best, ms = p1.autotune(cache, steps=2)
    say(f"  best: P={best.cols_per_lane} wpb={best.waves_per_block} persistent={best.persistent} "
        f"cap={best.waves_per_cu} chunked={best.chunked} align={best.band_align} {ms:.4f} ms")
    assert ms > 0 and open(cache).read().count("\n") == 1
    p2 = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
                  reals=reals, dt=0.05, tol=1e-7)
    best2, ms2 = p2.autotune(cache, steps=2)
    assert (best2.cols_per_lane, best2.waves_per_block, best2.persistent, best2.chunked, best2.band_align) == \
        (best.cols_per_lane, best.waves_per_block, best.persistent, best.chunked, best.band_align)
    assert open(cache).read().count("\n") == 1
    ref = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
                   reals=reals, dt=0.05, tol=1e-7)
    for p in (p1, ref):
        p.init_product_state([30, 31])
        p.propagate(10)
    assert np.array_equal(p1.state_numpy(), ref.state_numpy())


def test_boson_kernel_matches_distinguishable_symmetrised():
    """Two independent layouts: the triangle kernel and the full-grid kernel
    started from the symmetrised state must agree."""
    say("case: boson triangle vs full grid with symmetric start, N=90")
    reals = random_reals([90], seed=9)
    pb = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype="c128",
                  reals=reals, dt=0.05, tol=1e-14, sites=[30, 60])
    pd = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c128",
                  reals=reals, dt=0.05, tol=1e-14)
    full0 = np.zeros((90, 90), np.complex128)
    full0[30, 60] = full0[60, 30] = 1 / math.sqrt(2)
    pd.set_state_numpy(full0.reshape(-1))
    pb.propagate(40)
    pd.propagate(40)
    tri = pb.state_numpy()
    full = pd.state_numpy().reshape(90, 90)
    iu = np.triu_indices(90)
    assert np.max(np.abs(full[iu] - tri)) < 1e-12
    assert np.max(np.abs(full - full.T)) < 1e-12


# ------------------------------------------------------------- complex64

C64_BARS = {"kahan": 2e-7, "plain": 1e-6}   # amplitude bars after 200 steps (about 2.5x the measured errors)


@pytest.mark.parametrize("acc", ["kahan", "plain"])
def test_c64_against_oracle(acc):
    """complex64 state, FP32 stencil: max-abs amplitude error against the
    FP64 exact evolution after 200 steps of dt = 0.05 stays below 2e-7 with
    the compensated sum (measured 7.9e-8 / 8.2e-8) and 1e-6 with plain
    summation (measured 4.8e-7 / 3.0e-7), so a compensated sum that lost
    its compensation fails its bar; the measured error is printed."""
    say(f"case: c64 {acc} m=2 dist N=[64,100] and bosons N=70, 200 steps")
    for stat, Ns in (("distinguishable", [64, 100]), ("boson", [70])):
        reals = random_reals(Ns, seed=10)
        sb = B.BOSON if stat == "boson" else B.DISTINGUISHABLE
        plan = gpu_plan(m=2, statistics=stat, boundary="open", interaction="onsite", dtype="c64",
                        accumulation=acc, reals=reals, dt=0.05, tol=1e-7, sites=[30, 33])
        plan.propagate(200)
        err = compare_final(plan, reals, 2, sb, "open", "onsite", [30, 33], 10.0, C64_BARS[acc])
        n2, _ = plan.realization_norms()
        say(f"  {stat} {acc}: err {err:.3e}, |norm-1| max {np.max(np.abs(np.sqrt(n2) - 1)):.2e}")
        assert np.max(np.abs(np.sqrt(n2) - 1)) < (3e-7 if acc == "kahan" else 5e-6)


def test_compensated_sum_against_plain():
    """Rounding of the Taylor sum in complex64: 400 steps at a fixed order 7
    against the oracle's FP64 map of the same order (so that truncation
    cancels and only rounding is left).  The compensated sum keeps the norm
    drift and the amplitude error below those of plain summation (an FP32
    emulation of both sums predicts about 13x less norm drift and 2x less
    amplitude error)."""
    N, steps, dt = 48, 400, 0.05
    g = np.random.default_rng(21)
    reals = [(N, 1 + 0.1 * g.standard_normal(N - 1), np.zeros(N), 3.0) for _ in range(2)]
    say(f"case: compensated vs plain sum, N={N}, {steps} steps, order 7")
    res = {}
    for acc in ("kahan", "plain"):
        plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
                        accumulation=acc, reals=reals, dt=dt, order=7, sites=[N // 2 - 1, N // 2])
        plan.propagate(steps)
        psi = plan.state_numpy()
        err, drift = 0.0, 0.0
        for r, (n, J, eps, U) in enumerate(reals):
            H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", "onsite", J, eps, U)
            ref, _, _ = P.evolve_taylor(H, B.product_state(N, [N // 2 - 1, N // 2]), dt, steps, order=7)
            got = gpu_to_oracle(psi[r * N * N:(r + 1) * N * N], N, 2, B.DISTINGUISHABLE)
            err = max(err, float(np.max(np.abs(got - ref))))
            drift = max(drift, abs(float(np.vdot(got, got).real) - float(np.vdot(ref, ref).real)))
        res[acc] = (err, drift)
        say(f"  {acc}: amplitude error {err:.2e}, norm drift {drift:.2e}")
    assert res["kahan"][0] < 1e-6 and res["plain"][0] < 2e-6
    assert res["kahan"][1] < 0.5 * res["plain"][1]
    assert res["kahan"][0] < res["plain"][0]


# ------------------------------------------------------ monitoring / errors

def test_norm_alarm_raised_from_corrupted_state():
    """A host-corrupted state (one amplitude doubled) trips the FP64 norm
    alarm; the numerical error is reported by propagate."""
    from paper_1612_00746_amd import CtqwError
    say("case: norm alarm")
    reals = random_reals([20], seed=11)
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite",
                    dtype="c128", reals=reals, dt=0.05, tol=1e-14, norm_alarm=1e-6, sites=[5, 6])
    plan.propagate(3)
    psi = plan.state_numpy()
    psi[5 * 20 + 6] *= 2.0
    plan.set_state_numpy(psi)
    with pytest.raises(CtqwError) as e:
        plan.propagate(1)
    assert e.value.status == 6
    assert plan.stats().flags & 2


def test_renormalize_keeps_unit_norm_and_fixed_order_matches_oracle_taylor():
    """Fixed order n = 2 (a deliberately short series, as in Alg. 3 with a
    fixed n) drifts in norm; renormalisation rescales every step.  Without
    renormalisation the GPU must equal the oracle's fixed-order Taylor map."""
    say("case: fixed order 2, renormalize on/off")
    reals = random_reals([30], seed=12)
    N, J, eps, U = reals[0]
    H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", "onsite", J, eps, U)
    psi_o, _, _ = P.evolve_taylor(H, B.product_state(N, [10, 12]), 0.02, 50, order=2)
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c128",
                    reals=reals, dt=0.02, order=2, tol=0.0, sites=[10, 12])
    plan.propagate(50)
    assert np.max(np.abs(plan.state_numpy() - psi_o)) < 1e-13
    pr = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c128",
                  reals=reals, dt=0.02, order=2, tol=0.0, renormalize=True, sites=[10, 12])
    pr.propagate(50)
    assert abs(np.linalg.norm(pr.state_numpy()) - 1) < 1e-13
    ref = psi_o / np.linalg.norm(psi_o)
    # renormalising every step equals renormalising once at the end (linear map)
    assert np.max(np.abs(pr.state_numpy() - ref)) < 1e-12


def test_zero_steps_and_observe():
    say("case: zero steps / observe at t=0")
    reals = random_reals([12, 12], seed=13)
    plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype="c64",
                    reals=reals, dt=0.05, tol=1e-7, sites=[3, 3])
    out = plan.propagate(0, 1, 1)
    assert out.shape == (1, 12)
    expect = np.zeros(12)
    expect[3] = 2.0
    assert np.max(np.abs(out[0] - expect)) < 1e-7
    assert np.max(np.abs(plan.observe(1) - expect)) < 1e-7


# ------------------------------------------------------------ launch shapes
# Each shape runs in its own test; all must be bitwise identical to the
# regular one-column-per-lane launch (the arithmetic of an amplitude does not
# depend on the band partition, the columns per lane or the launch form).

_SHAPE_REALS = None


def _shape_state(launch):
    # 520 sites: several bands at either width, the last one past the chain's end
    reals = random_reals([100, 200, 37, 520], seed=8)
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite",
                    dtype="c64", reals=reals, dt=0.05, tol=1e-7, launch=launch, sites=[30, 31])
    plan.propagate(25)
    return plan.state_numpy()


@pytest.mark.parametrize("launch", [
    {"cols_per_lane": 2},
    {"cols_per_lane": 1, "waves_per_block": 1},
    {"cols_per_lane": 1, "persistent": 1},
    {"cols_per_lane": 2, "persistent": 1, "waves_per_block": 1},
    {"cols_per_lane": 1, "persistent": 1, "waves_per_cu": 8},
    {"cols_per_lane": 1, "band_align": 0},
    {"cols_per_lane": 2, "band_align": 64},
    {"cols_per_lane": 2, "persistent": 1, "band_align": 0},
    {"cols_per_lane": 1, "band_mode": 1},
    {"cols_per_lane": 2, "band_mode": 1},
    {"cols_per_lane": 2, "persistent": 1, "waves_per_block": 1, "band_mode": 1},
    {"cols_per_lane": 1, "row_segments": 0},
    {"cols_per_lane": 2, "row_segments": 3},
    {"cols_per_lane": 1, "persistent": 1, "row_segments": 16},
], ids=["P2", "P1-wpb1", "P1-persistent", "P2-persistent-wpb1", "P1-persistent-cap8", "P1-unaligned",
        "P2-align64", "P2-persistent-unaligned", "P1-window-aligned", "P2-window-aligned",
        "P2-persistent-window-aligned", "P1-row-segments-auto", "P2-row-segments-3",
        "P1-persistent-row-segments-16"])
def test_launch_shape_bitwise_identical(launch):
    """Bitwise identical whatever the block shape, launch form, band
    boundaries or columns per lane: the complex64 full-grid stencil is one
    fixed sequence of FMAs per amplitude (a column computed in two bands'
    halos, or by a lane holding one or two columns, follows the same
    arithmetic)."""
    say(f"case: launch shape {launch} vs regular with the same columns per lane")
    P_ = launch.get("cols_per_lane", 1)
    launch = {"row_segments": 1, **launch}
    ref = _shape_state({"cols_per_lane": P_, "row_segments": 1})
    got = _shape_state(launch)
    assert np.array_equal(got, ref)
    if P_ == 2:
        assert np.array_equal(got, _shape_state({"cols_per_lane": 1, "row_segments": 1}))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("statistics,boundary,interaction", [
    ("distinguishable", "open", "onsite"),
    ("boson", "open", "onsite"),
    ("fermion", "open", "nearest"),
    ("distinguishable", "periodic", "onsite"),
    ("distinguishable", "periodic", "nearest"),
])
def test_row_segments_match_the_unsplit_sweep(statistics, boundary, interaction, dtype):
    """Splitting a band's rows into segments (each swept from a halo of
    Taylor-order rows before its first output row to as many after its
    last) computes every amplitude from the same neighbours with the same
    coefficients.  The complex64 full-grid stencil is one fixed sequence of
    FMAs, so there the state is bitwise unchanged; the compiler-generated
    stencils (triangle, complex128) may contract a row's products
    differently at another position of the unrolled sweep, so there the
    states agree to rounding (measured: a few units in the last place of
    the smallest amplitudes).  Both runs match the FP64 oracle."""
    say(f"case: row segments {statistics} {boundary} {interaction} {dtype}")
    reals = random_reals([100, 37, 150], boundary=boundary, seed=21)
    n_steps, dt, sites = 12, 0.05, [17, 30]

    def run(seg):
        plan = gpu_plan(m=2, statistics=statistics, boundary=boundary, interaction=interaction, dtype=dtype,
                        reals=reals, dt=dt, tol=1e-7 if dtype == "c64" else 1e-12,
                        launch={"row_segments": seg}, sites=sites)
        items = plan.work_items()[0]
        plan.propagate(n_steps)
        return items, plan.state_numpy(), plan.realization_norms(), plan.orders(), plan.layout()

    n1, ref, (lo1, hi1), orders, off = run(1)
    exact = dtype == "c64" and statistics == "distinguishable"
    for seg in (0, 5):
        n, got, (lo, hi), _, _ = run(seg)
        d = np.max(np.abs(got.astype(np.complex128) - ref.astype(np.complex128)))
        say(f"  row_segments={seg}: {n} items (unsplit {n1}), max |split - unsplit| = {d:.3e}")
        assert n > n1
        if exact:
            assert np.array_equal(got, ref)
        else:
            assert d <= (1e-6 if dtype == "c64" else 1e-13) * np.max(np.abs(ref))
        # squared norms in FP64; the last term's squares are summed in the
        # state's precision per segment before widening
        assert np.allclose(lo, lo1, rtol=1e-12 if exact or dtype == "c128" else 1e-7, atol=0)
        assert np.allclose(hi, hi1, rtol=1e-5 if dtype == "c64" else 1e-12, atol=1e-300)
    # the split run against the oracle's map of the same orders
    for r, (N, J, eps, U) in enumerate(reals):
        H = oracle_H(N, 2, statistics, boundary, interaction, J, eps, U)
        c, _, _ = P.evolve_taylor(H, B.product_state(N, sites, statistics), dt, n_steps, order=int(orders[r]))
        g = gpu_to_oracle(got[off[r]:off[r + 1]], N, 2, statistics)
        err = np.max(np.abs(g - c))
        say(f"  r={r} N={N}: split run vs oracle map {err:.2e}")
        assert err <= (2e-6 if dtype == "c64" else 1e-12)
