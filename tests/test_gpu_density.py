"""GPU parity of the ensemble-averaged density matrix (Eq. 2): the library
gathers each lattice-size group's states and forms rho = A A^H / R_g with
one Hermitian rank-R_g update on the matrix cores; the oracle sums
|psi_r><psi_r| over its own exactly evolved states."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import observables as O
from oracle import propagate as P

from _helpers import gpu_plan, oracle_H, say

pytestmark = pytest.mark.gpu


def reals_for(Ns, seed):
    g = np.random.default_rng(seed)
    return [(N, 1 + 0.1 * g.standard_normal(N - 1), g.uniform(-0.3, 0.3, N), float(g.uniform(0.5, 2.0))) for N in Ns]


def oracle_rho(reals, sb, sites, t):
    rhos = {}
    for N in sorted({r[0] for r in reals}):
        states = []
        for (n, J, eps, U) in reals:
            if n != N:
                continue
            H = oracle_H(N, 2, sb, "open", "onsite", J, eps, U)
            states.append(P.EDPropagator(H).evolve(B.product_state(N, sites, sb), t))
        rhos[N] = O.density_matrix(states)
    return rhos


@pytest.mark.parametrize("stat", ["distinguishable", "boson"])
def test_density_matrix_c128_against_the_oracle(stat):
    """Uneven batch (two lattice sizes, two groups), complex128, t = 1:
    every group's density matrix within 1e-10 of the oracle's, Hermitian
    with unit trace."""
    sb = B.BOSON if stat == "boson" else B.DISTINGUISHABLE
    reals = reals_for([14, 11, 14, 11, 14], 31)
    sites = [4, 6]
    dt, steps = 0.02, 50
    say(f"case: density matrix c128 {stat}, N={[r[0] for r in reals]}, t={dt * steps}")
    plan = gpu_plan(m=2, statistics=stat, boundary="open", interaction="onsite", dtype="c128", reals=reals,
                    dt=dt, tol=1e-14, sites=sites)
    plan.propagate(steps)
    ref = oracle_rho(reals, sb, sites, dt * steps)
    for gidx, N in enumerate(plan.groups()):
        rho = plan.density_matrix(gidx).cpu().numpy()
        err = float(np.max(np.abs(rho - ref[int(N)])))
        say(f"  group {gidx} (N={N}, D={rho.shape[0]}): max |rho - oracle| = {err:.2e}, trace {np.trace(rho).real:.15f}")
        assert err <= 1e-10
        assert np.allclose(rho, rho.conj().T, atol=1e-15)
        assert abs(np.trace(rho) - 1) < 1e-12


def test_density_matrix_c64_lower_triangle():
    """complex64: the full matrix within 1e-6 of the oracle's; with
    lower_only the lower triangle is the same and the upper stays zero."""
    reals = reals_for([20] * 6, 32)
    sites = [9, 10]
    dt, steps = 0.05, 40
    say("case: density matrix c64, N=20, R=6, lower triangle")
    plan = gpu_plan(m=2, statistics="distinguishable", boundary="open", interaction="onsite", dtype="c64",
                    reals=reals, dt=dt, tol=1e-7, sites=sites)
    plan.propagate(steps)
    ref = oracle_rho(reals, B.DISTINGUISHABLE, sites, dt * steps)[20]
    full = plan.density_matrix(0).cpu().numpy().astype(np.complex128)
    low = plan.density_matrix(0, lower_only=True).cpu().numpy().astype(np.complex128)
    err = float(np.max(np.abs(full - ref)))
    say(f"  max |rho - oracle| = {err:.2e}")
    assert err <= 1e-6
    il = np.tril_indices(full.shape[0])
    iu = np.triu_indices(full.shape[0], 1)
    assert np.array_equal(low[il], full[il])
    assert np.all(low[iu] == 0)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("stat,N,R", [("boson", 23, 37), ("distinguishable", 19, 21), ("fermion", 25, 17)])
def test_density_matrix_ragged_tiles(dtype, stat, N, R):
    """Dimensions that are not whole tiles (D = 276, 361, 325 against 64 /
    128-row tiles) and realisation counts that are not whole stages: the
    full matrix and the lower triangle against the oracle's sum of
    |psi><psi| of its exactly evolved states (fermions: embedded in the
    triangle basis, whose diagonal rows and columns are zero)."""
    sb = {"boson": B.BOSON, "distinguishable": B.DISTINGUISHABLE, "fermion": B.FERMION}[stat]
    reals = reals_for([N] * R, 33)
    sites = [N // 2 - 2, N // 2 + 1]
    dt, steps = 0.05, 30
    say(f"case: density matrix {dtype} {stat} N={N} R={R} (ragged tiles and stages)")
    plan = gpu_plan(m=2, statistics=stat, boundary="open", interaction="onsite", dtype=dtype, reals=reals,
                    dt=dt, tol=1e-14 if dtype == "c128" else 1e-7, sites=sites)
    plan.propagate(steps)
    states = []
    for (n, J, eps, U) in reals:
        H = oracle_H(N, 2, sb, "open", "onsite", J, eps, U)
        c = P.EDPropagator(H).evolve(B.product_state(N, sites, sb), dt * steps)
        if sb == B.FERMION:           # the triangle basis: zero on the diagonal states
            tri = B.basis_states(N, 2, B.BOSON)
            full = np.zeros(len(tri), dtype=np.complex128)
            full[tri[:, 0] < tri[:, 1]] = c
            c = full
        states.append(c)
    ref = O.density_matrix(states)
    rho = plan.density_matrix(0).cpu().numpy().astype(np.complex128)
    low = plan.density_matrix(0, lower_only=True).cpu().numpy().astype(np.complex128)
    err = float(np.max(np.abs(rho - ref)))
    bar = 1e-12 if dtype == "c128" else 2e-6
    say(f"  D={rho.shape[0]}: max |rho - oracle| = {err:.2e} (bar {bar:.0e})")
    assert err <= bar
    il = np.tril_indices(rho.shape[0])
    iu = np.triu_indices(rho.shape[0], 1)
    assert np.array_equal(low[il], rho[il]) and np.all(low[iu] == 0)
    assert np.array_equal(rho, rho.conj().T)


def test_density_matrix_full_two_boson_workload_sampled():
    """The two-boson workload's shape (1000 realisations, N = 128, D = 8256,
    complex64) from seeded random states set on the device: 2000 sampled
    entries of rho (both triangles, diagonal included) against their
    definition (1/R) sum_r c_ri conj(c_rj) evaluated in FP64 from the same
    states, and the trace."""
    import math
    import torch
    from workloads import C2
    w = C2("c64")
    reals = w.all_realizations()
    say("case: density matrix at the two-boson workload's shape, sampled entries")
    plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype="c64", reals=reals,
                    dt=w.dt, tol=w.tol, sites=list(w.start))
    D = w.N * (w.N + 1) // 2
    g = np.random.default_rng(77)
    phi = (g.standard_normal((w.R, D)) + 1j * g.standard_normal((w.R, D))).astype(np.complex64)
    phi /= np.linalg.norm(phi, axis=1, keepdims=True).astype(np.float32)
    plan.set_state_numpy(phi.reshape(-1))
    rho = plan.density_matrix(0)
    torch.cuda.synchronize()
    tri = B.basis_states(w.N, 2, B.BOSON)
    c = phi.astype(np.complex128) * np.where(tri[:, 0] < tri[:, 1], math.sqrt(2.0), 1.0)
    i = g.integers(0, D, 2000)
    j = g.integers(0, D, 2000)
    i[:50] = j[:50]
    got = rho[torch.from_numpy(i).cuda(), torch.from_numpy(j).cuda()].cpu().numpy().astype(np.complex128)
    want = np.einsum("ri,ri->i", c[:, i], np.conj(c[:, j])) / w.R
    err = float(np.max(np.abs(got - want)))
    say(f"  max |rho_ij - definition| over 2000 entries = {err:.2e}; trace {float(torch.trace(rho).real):.7f}")
    assert err <= 1e-8
