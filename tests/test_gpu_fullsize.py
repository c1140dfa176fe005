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
C64_BAR = 2e-5   # complex64 amplitude bar against the FP64 map (derivation: DESIGN, parity bars)


def test_c3_full_size_sampled_against_the_oracle():
    import torch
    import bench
    from workloads import C3

    w = C3("c64")
    launch = dict(cols_per_lane=2, persistent=1, waves_per_block=1, waves_per_cu=8, use_graph=1, band_align=128)
    say(f"case: C3 full size, c64 Kahan, {STEPS} steps, launch {launch}")
    plan = bench.build_plan(w, "c64", "kahan", launch, w.tol)
    sizes = w.lattice_sizes()
    orders = plan.orders()
    plan.propagate(STEPS)

    n2, _ = plan.realization_norms()
    drift = float(np.max(np.abs(np.sqrt(n2) - 1.0)))
    say(f"  max |norm - 1| over {w.R} realisations: {drift:.2e}")
    assert drift < 1e-6

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
