"""The batched complex64 workload at its full size (4096 realisations of two
distinguishable walkers, N_r in {64, 96, ..., 1024}, 1.54e9 amplitudes), in
the launch configuration the benchmark times (two columns per lane,
persistent grid, one wave per block, 128-byte band boundaries, captured step
loop; orders 6 and 7 in one launch).  Sampled realisations — the smallest
and the largest chain among them — are checked one by one against the
oracle's FP64 Taylor map at each realisation's own a-priori order; the
properties that hold at any size (unit FP64 norms, occupations summing to
the particle number) are checked on the whole batch."""

import ctypes as C

import numpy as np
import pytest

from oracle import basis as B
from oracle import propagate as P

from _helpers import gpu_to_oracle, oracle_H, reference_order, say

pytestmark = pytest.mark.gpu

STEPS = 20
# complex64 amplitude bar against the FP64 map of the same order after 20
# steps: about 2x the largest measured error (5e-8 to 9e-8, mostly the FP32
# rounding of the dt-scaled couplings); the norms of all realisations are
# held to 5e-7 of 1 (measured 1.9e-7) and the occupation sums to 1e-5 of 2.
C64_BAR = 2e-7


@pytest.mark.parametrize("band_mode", [0, 1], ids=["output-aligned", "window-aligned"])
def test_c3_full_size_sampled_against_the_oracle(band_mode):
    import torch
    import bench
    from workloads import C3

    w = C3("c64")
    launch = dict(cols_per_lane=2, persistent=1, waves_per_block=1, waves_per_cu=8, use_graph=1, band_align=128,
                  band_mode=band_mode)
    say(f"case: C3 full size, c64 Kahan, {STEPS} steps, launch {launch}")
    plan = bench.build_plan(w, "c64", "kahan", launch, w.tol)
    sizes = w.lattice_sizes()
    orders = plan.orders()
    plan.propagate(STEPS)

    n2, _ = plan.realization_norms()
    drift = float(np.max(np.abs(np.sqrt(n2) - 1.0)))
    say(f"  max |norm - 1| over {w.R} realisations: {drift:.2e}")
    assert drift < 5e-7

    occ = plan.observe(1)
    groups = plan.groups()
    total, o = [], 0
    for N in groups:
        total.append(float(np.sum(occ[o:o + N])))
        o += N
    say(f"  occupation sums per group: min {min(total):.7f} max {max(total):.7f} ({len(groups)} groups)")
    assert np.allclose(total, 2.0, atol=1e-5)

    # the state, copied on the device; only the sampled realisations come to the host
    state_bytes, _ = plan.sizes()
    dev = torch.empty(state_bytes, dtype=torch.uint8, device="cuda")
    assert plan.lib.ctqw_get_state(plan.h, C.c_void_p(dev.data_ptr()), 1) == 0
    psi = dev.view(torch.complex64)
    off = plan.layout()
    g = np.random.default_rng(2024)
    sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), *g.choice(w.R, 4, replace=False).tolist()})
    for r in sample:
        N, J, eps, U = w.all_realizations([r])[0]
        n_r = reference_order(J, eps, U, 2, w.dt, w.tol)
        assert orders[r] == n_r
        got = gpu_to_oracle(psi[off[r]:off[r + 1]].cpu().numpy(), N, 2, B.DISTINGUISHABLE)
        H = oracle_H(N, 2, B.DISTINGUISHABLE, "open", "onsite", J, eps, U)
        psi0 = B.product_state(N, w.start_sites(N), B.DISTINGUISHABLE)
        ref, _, _ = P.evolve_taylor(H, psi0, w.dt, STEPS, order=n_r)
        err = float(np.max(np.abs(got - ref)))
        say(f"  r={r} N={N} order {n_r}: max |psi - oracle| = {err:.2e}")
        assert err <= C64_BAR


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_c2_full_configuration_sampled_against_the_oracle(dtype):
    """The two-boson workload at its stated configuration: 1000
    realisations on N = 128 (D = 8256 each), on-site U = 2, J ~ N(1, 0.2^2),
    eps ~ U[-0.5, 0.5], 1000 steps of dt = 0.05 to t = 50, with the ensemble
    occupation output every 20 steps.  Six sampled realisations are
    compared amplitude by amplitude with the oracle's Taylor route at
    tolerance 1e-15 (within steps x 1e-15 of the exact evolution), and the
    final ensemble occupation of the sample with the oracle's.  complex128:
    1e-10.  complex64 (tolerance 1e-7, compensated sum) splits its error in
    two.  Representation: the kernels hold dt*J, dt*eps and dt*U in FP32 and
    form each diagonal entry as an FP32 sum of them, i.e. they evolve with a
    Hamiltonian H32 that differs from H by rounding alone; the oracle
    evolves the sample with H32 too, and |psi_H32 - psi_H| (measured
    0.3e-6 to 1.0e-6) is a property of FP32 storage, not of the kernels.
    Arithmetic: against the oracle's H32 evolution the kernels may differ
    by their roundings only: one rounding of each component of the state
    per step (2^-24 relative) plus the rounding of the summed terms, at
    |psi| <= 0.3, accumulating as a random walk over 1000 steps:
    sqrt(1000) * 1.2 * 6e-8 * 0.3 = 7e-7, held to 1.5e-6.  So the bars are
    amplitude <= 1.5e-6 against the H32 evolution and <= |psi_H32 - psi_H|
    + 1.5e-6 against the exact one; occupation 1e-6 and |norm - 1| 1e-6."""
    import torch
    from oracle import observables as O
    from workloads import C2
    w = C2(dtype)
    say(f"case: C2 full configuration {dtype}: R={w.R} N={w.N} {w.n_steps} steps")
    reals = w.all_realizations()
    from _helpers import gpu_plan
    plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype=dtype, reals=reals,
                    dt=w.dt, tol=w.tol, observables=1, sites=list(w.start))
    out = plan.propagate(w.n_steps, w.output_every, 1)
    assert out.shape[0] == w.n_steps // w.output_every + 1
    n2, _ = plan.realization_norms()
    drift = float(np.max(np.abs(np.sqrt(n2) - 1.0)))
    assert np.allclose(out[:, :w.N].sum(axis=1), 2.0, atol=1e-9 if dtype == "c128" else 1e-5)
    orders = plan.orders()
    state_bytes, _ = plan.sizes()
    dev = torch.empty(state_bytes, dtype=torch.uint8, device="cuda")
    assert plan.lib.ctqw_get_state(plan.h, C.c_void_p(dev.data_ptr()), 1) == 0
    psi = dev.view(torch.complex128 if dtype == "c128" else torch.complex64)
    off = plan.layout()
    sample = sorted(np.random.default_rng(50).choice(w.R, 6, replace=False).tolist())
    st = B.basis_states(w.N, 2, B.BOSON)
    worst, worst32, excess, occ_o, occ_g = 0.0, 0.0, -1.0, [], []
    for r in sample:
        N, J, eps, U = reals[r]
        H = oracle_H(N, 2, B.BOSON, "open", "onsite", J, eps, U)
        psi0 = B.product_state(N, list(w.start), B.BOSON)
        ref, _, _ = P.evolve_taylor(H, psi0, w.dt, w.n_steps, tol=1e-15)
        got = gpu_to_oracle(psi[off[r]:off[r + 1]].cpu().numpy(), N, 2, B.BOSON)
        err = float(np.max(np.abs(got - ref)))
        worst = max(worst, err)
        if dtype == "c64":
            ref32, _, _ = P.evolve_taylor(fp32_boson_onsite_H(N, J, eps, U, w.dt, st), psi0, w.dt, w.n_steps,
                                          tol=1e-15)
            rep = float(np.max(np.abs(ref32 - ref)))
            e32 = float(np.max(np.abs(got - ref32)))
            worst32 = max(worst32, e32)
            excess = max(excess, err - rep)
            say(f"  r={r}: |psi - oracle| {err:.2e}, |psi - oracle(H32)| {e32:.2e}, "
                f"|oracle(H32) - oracle| {rep:.2e}")
        occ_o.append(O.occupation(ref, st, N))
        occ_g.append(O.occupation(got, st, N))
    e_occ = float(np.max(np.abs(O.ensemble_mean(occ_g) - O.ensemble_mean(occ_o))))
    say(f"  orders {int(orders.min())}-{int(orders.max())}; sample {sample}: amplitude {worst:.2e}"
        + (f" (against the H32 evolution {worst32:.2e}, beyond the representation {excess:.2e})"
           if dtype == "c64" else "")
        + f", occupation {e_occ:.2e}, max |norm - 1| over all {w.R}: {drift:.2e}")
    if dtype == "c128":
        assert worst <= 1e-10 and e_occ <= 1e-10 and drift <= 1e-10
    else:
        assert worst32 <= 1.5e-6 and excess <= 1.5e-6 and e_occ <= 1e-6 and drift <= 1e-6


def fp32_boson_onsite_H(N, J, eps, U, dt, states):
    """The two-boson on-site Hamiltonian as FP32 tables of dt-scaled
    parameters represent it: hoppings fl(dt J)/dt, diagonal entries
    fl(fl(dt eps_a) + fl(dt eps_b)) (plus fl(dt U), rounded again, on a
    doubly occupied node) over dt."""
    import scipy.sparse as sp
    f32 = lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)
    Jr = f32(np.asarray(J) * dt) / dt
    Er = f32(np.asarray(eps) * dt)
    H = oracle_H(N, 2, B.BOSON, "open", "onsite", Jr, np.zeros(N), 0.0)
    d = f32(Er[states[:, 0]] + Er[states[:, 1]])
    d = np.where(states[:, 0] == states[:, 1], f32(d + f32(U * dt)), d)
    return (H - sp.diags(H.diagonal()) + sp.diags(d / dt)).tocsr()


def test_c4_full_lattice_gradient_against_the_oracle():
    """The gradient workload's lattice at full size (two bosons on N = 256,
    U = 1, start (191, 192), loss = probability that both are in nodes
    192..255 after 400 steps of dt = 0.05, checkpoints every 32) on a subset
    of two realisations, complex128: the loss equals the oracle's
    truncated-Taylor loss at the same order (1e-12) and the adjoint's
    derivative along a random direction of (Jbar, epsbar) matches the
    central difference of the oracle's loss (1e-6 relative)."""
    from oracle import gradients as Gr
    from workloads import C4
    from _helpers import gpu_plan
    w = C4("c128")
    R = 2
    say(f"case: C4 full lattice N={w.N}, R={R}, {w.n_steps} steps, c128 gradient vs oracle")
    reals = w.all_realizations(range(R))
    plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype="c128", reals=reals,
                    dt=w.dt, tol=w.tol, sites=list(w.start))
    order = int(plan.orders().max())
    sw = (np.arange(w.N) >= 192).astype(float)
    loss, gJ, gE = plan.gradient(w.n_steps, 32, sw, "product")
    dJ = np.array([w.noise_only(r)[0] for r in range(R)])
    dE = np.array([w.noise_only(r)[1] for r in range(R)])
    U = np.array([r[3] for r in reals])
    ens = Gr.Ensemble(w.N, 2, B.BOSON, dJ, dE, U, list(w.start))
    wts = Gr.diagonal_weights(ens.states, sw, Gr.PRODUCT)
    Jbar, epsbar = np.full(w.N - 1, w.Jbar), np.full(w.N, w.epsbar)
    fn = lambda a, b: Gr.loss_taylor(ens, a, b, wts, w.dt, w.n_steps, order)  # noqa: E731
    l0 = fn(Jbar, epsbar)
    rs = np.random.default_rng(9)
    vJ, vE = rs.normal(size=w.N - 1), rs.normal(size=w.N)
    fd = Gr.fd_directional(fn, Jbar, epsbar, vJ, vE, h=1e-5)
    ad = float(gJ @ vJ + gE @ vE)
    say(f"  order {order}: loss {loss:.12e} (oracle {l0:.12e}); directional adjoint {ad:.10e} vs oracle FD {fd:.10e}")
    assert abs(loss - l0) <= 1e-12
    assert abs(ad - fd) <= 1e-6 * abs(fd)


def test_c5_full_run_length_properties_and_sampled_realisations():
    """The three-walker workload at its stated configuration: 64
    realisations on N = 256 (16.8M amplitudes each, 1.07e9 in all),
    nearest-neighbour U = 1, eps ~ U[-1, 1], J = 1, dt = 0.02, tolerance
    1e-7, complex64, 500 steps to t = 10 with the ensemble occupation and
    pair correlation every 50 steps, in the product form the benchmark
    times.  No oracle evolves a 16.8M-amplitude state within a test, so the
    whole batch is held to properties that hold at any size:
      * at every output the ensemble occupation sums to m = 3 and the pair
        correlation (ordered pairs a != b) to m(m - 1) = 6, within 1e-5;
      * every realisation's FP64 norm stays within 5e-6 of 1 (FP32 rounding
        of the state, one per pass, as a random walk over 1000 passes);
      * the light cone: a walker started at 127..129 reaches a node d hops
        away only through d of its own hops, each of norm 2J, so its
        amplitude there is at most (2Jt)^d e^(2Jt) / d!, below 1e-19 for
        d >= 100 at t = 10: the ensemble occupation of nodes 0..27 and
        229..255 stays below 1e-12.
    Two sampled realisations (the first and the last) are run alone in
    complex128 with chained passes at the same order (that form is held to
    1e-12 of the oracle on smaller lattices) and every complex64 amplitude
    is within 2e-6 of them: the FP32 rounding of the state (6e-8 per
    component and pass, a random walk over 1000 passes) plus the FP32
    representation of the dt-scaled couplings (a Hamiltonian that differs
    by about 6e-8 relative, acting for t = 10)."""
    import torch
    from workloads import C5
    from _helpers import gpu_plan
    w = C5()
    say(f"case: C5 full configuration c64: R={w.R} N={w.N} {w.n_steps} steps, product form")
    reals = w.all_realizations()
    plan = gpu_plan(m=3, statistics="distinguishable", boundary="open", interaction="nearest", dtype="c64",
                    reals=reals, dt=w.dt, tol=w.tol, observables=3, sites=list(w.start),
                    launch={"three_form": 1})
    out = plan.propagate(w.n_steps, w.output_every, 3)
    N = w.N
    assert out.shape == (w.n_steps // w.output_every + 1, N + N * N)
    occ_sum = out[:, :N].sum(axis=1)
    pair_sum = out[:, N:].sum(axis=1)
    n2, _ = plan.realization_norms()
    drift = float(np.max(np.abs(np.sqrt(n2) - 1.0)))
    far = float(np.max(np.concatenate([out[:, :28], out[:, 229:N]], axis=1)))
    order = int(plan.orders().max())
    state_bytes, _ = plan.sizes()
    dev = torch.empty(state_bytes, dtype=torch.uint8, device="cuda")
    assert plan.lib.ctqw_get_state(plan.h, C.c_void_p(dev.data_ptr()), 1) == 0
    psi = dev.view(torch.complex64)
    off = plan.layout()
    sample = [0, w.R - 1]
    got = [psi[off[r]:off[r + 1]].cpu().numpy().astype(np.complex128) for r in sample]
    del plan, dev, psi
    torch.cuda.empty_cache()
    ref_plan = gpu_plan(m=3, statistics="distinguishable", boundary="open", interaction="nearest",
                        dtype="c128", reals=[reals[r] for r in sample], dt=w.dt, order=order,
                        sites=list(w.start), launch={"three_form": 0})
    ref_plan.propagate(w.n_steps)
    ref = ref_plan.state_numpy()
    D = N ** 3
    diff = max(float(np.max(np.abs(got[k] - ref[k * D:(k + 1) * D]))) for k in range(len(sample)))
    say(f"  order {order}: occupation sums {occ_sum.min():.7f}..{occ_sum.max():.7f}, pair sums "
        f"{pair_sum.min():.7f}..{pair_sum.max():.7f}, max |norm - 1| {drift:.2e}, far occupation {far:.1e}, "
        f"sample {sample} against complex128 {diff:.2e}")
    assert np.allclose(occ_sum, 3.0, atol=1e-5) and np.allclose(pair_sum, 6.0, atol=1e-5)
    assert drift <= 5e-6
    assert far <= 1e-12
    assert diff <= 2e-6
