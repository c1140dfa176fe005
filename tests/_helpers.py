"""Shared test helpers: run the GPU path through the C ABI and the FP64 oracle
on the same seeded inputs, and map between their state layouts."""

from __future__ import annotations

import math
import sys

import numpy as np

from oracle import basis as B
from oracle import hamiltonian as Hm
from oracle import propagate as P


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gershgorin_x(J, eps, U, m, dt):
    """x = dt * G with G = m*max_i(|eps_i| + |J_{i-1}| + |J_i|) + |U| m(m-1)/2,
    the documented bound on ||H||_2 (Gershgorin; J padded with a zero bond
    for open chains)."""
    N = len(eps)
    Jp = np.zeros(N)
    Jp[:len(J)] = J
    G = m * max(abs(eps[i]) + abs(Jp[(i - 1) % N]) + abs(Jp[i]) for i in range(N))
    G += abs(U) * m * (m - 1) / 2
    return G * dt


def tail_bound(x, n):
    """Remainder factor of the truncated series: sum_{j>n} x^j/j! is at most
    x^n/n! * (x/(n+1)) / (1 - x/(n+2)) (geometric bound of the ratios)."""
    return (x / (n + 1)) / (1 - x / (n + 2)) if x < n + 2 else math.inf


def reference_order(J, eps, U, m, dt, tol, periodic=False):
    """Smallest n with x^(n+1)/(n+1)!/(1 - x/(n+2)) <= tol (documented rule)."""
    x = gershgorin_x(J, eps, U, m, dt)
    n = 1
    while True:
        b = x ** (n + 1) / math.factorial(n + 1) / (1 - x / (n + 2)) if x < n + 2 else math.inf
        if b <= tol:
            return n
        n += 1


def params_for(w, subset=None):
    """[(N, J, eps, U)] for realisations of a workload."""
    return w.all_realizations(subset)


def pack(reals):
    Ns = [r[0] for r in reals]
    J = np.concatenate([r[1] for r in reals])
    eps = np.concatenate([r[2] for r in reals])
    U = np.array([r[3] for r in reals], dtype=np.float64)
    return Ns, J, eps, U


def gpu_plan(*, m, statistics, boundary, interaction, dtype, reals, dt, tol=0.0, order=0,
             accumulation="kahan", observables=1, renormalize=False, norm_alarm=0.0, launch=None,
             sites=None):
    from paper_1612_00746_amd import Plan, make_problem
    Ns, J, eps, U = pack(reals)
    uniform = len(set(Ns)) == 1
    pr, keep = make_problem(m, len(Ns), Ns[0] if uniform else Ns, dt, statistics=statistics,
                            boundary=boundary, interaction=interaction, dtype=dtype,
                            accumulation=accumulation, taylor_order=order, taylor_tol=tol,
                            renormalize=renormalize, norm_alarm=norm_alarm, observables=observables)
    plan = Plan(pr)
    plan._keep.append(keep)
    if launch:
        plan.set_launch(**launch)
    plan.set_params(J, eps, U)
    plan.bind()
    if sites is not None:
        plan.init_product_state(sites)
    return plan


def oracle_H(N, m, statistics, boundary, interaction, J, eps, U):
    return Hm.hamiltonian(N, m, J, eps, U if m > 1 else 0.0, statistics, boundary, interaction)


def gpu_to_oracle(psi_r, N, m, statistics):
    """GPU layout of one realisation -> oracle basis coefficients.  The GPU
    stores phi(x1, x2) on x1 <= x2 for bosons and fermions (the fermions'
    diagonal is 0); the normalised basis coefficient is sqrt(2) phi off the
    diagonal (bosons: phi on it; fermions have no diagonal states)."""
    psi_r = np.asarray(psi_r, dtype=np.complex128)
    if m == 2 and statistics == B.BOSON:
        st = B.basis_states(N, 2, B.BOSON)
        return psi_r * np.where(st[:, 0] < st[:, 1], math.sqrt(2.0), 1.0)
    if m == 2 and statistics == B.FERMION:
        tri = B.basis_states(N, 2, B.BOSON)
        return psi_r[tri[:, 0] < tri[:, 1]] * math.sqrt(2.0)
    return psi_r


def oracle_to_gpu(c, N, m, statistics):
    c = np.asarray(c, dtype=np.complex128)
    if m == 2 and statistics == B.BOSON:
        st = B.basis_states(N, 2, B.BOSON)
        return c / np.where(st[:, 0] < st[:, 1], math.sqrt(2.0), 1.0)
    if m == 2 and statistics == B.FERMION:
        tri = B.basis_states(N, 2, B.BOSON)
        out = np.zeros(len(tri), dtype=np.complex128)
        out[tri[:, 0] < tri[:, 1]] = c / math.sqrt(2.0)
        return out
    return c


def gpu_tri_diagonal(psi_r, N):
    """The diagonal entries phi(x, x) of the triangle layout."""
    tri = B.basis_states(N, 2, B.BOSON)
    return np.asarray(psi_r)[tri[:, 0] == tri[:, 1]]
