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
