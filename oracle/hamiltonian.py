"""Sparse FP64 Hamiltonian of one noisy realisation (oracle, CPU).

Eq. (1) of the paper: H_ab is a deterministic part plus a stochastic part
when b = a or b is a neighbour of a, and zero otherwise; the diagonal holds
on-site energies and the off-diagonal entries the tunnelling amplitudes, with
equal rates for a->b and b->a (Sec. 2.2), so H is real symmetric.  With hbar
set to 1 all energies are in units of the hopping scale.

For one particle on an N-site chain this is the tridiagonal matrix H1 with
diagonal eps_i and H1[i, i+1] = H1[i+1, i] = +J_i for bond i (nodes i, i+1);
a periodic chain adds the bond N-1 between node N-1 and node 0.  The sign
+J is the one for which a single walker started on node s has amplitude
(-i)^n J_n(2Jt) on node s+n.

For m particles: H = sum_a (identity except H1 on particle a) + diag V,
where V counts interacting pairs,
    on-site:           V(x) = U * #{a<b : x_a == x_b}
    nearest-neighbour: V(x) = U * #{a<b : |x_a - x_b| == 1}
(the nearest-neighbour form uses the chain distance, also across the
periodic bond).  Bosons use H_S = S^T H S with S from ``basis.symmetrizer``,
fermions H_A = A^T H A with A from ``basis.antisymmetrizer``.

Test infrastructure only; see the package docstring.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import BOSON, DISTINGUISHABLE, FERMION, antisymmetrizer, basis_states, symmetrizer

OPEN = "open"
PERIODIC = "periodic"
ONSITE = "onsite"
NEAREST = "nearest"


def n_bonds(N: int, boundary: str) -> int:
    return N - 1 if boundary == OPEN else N


def single_particle(J, eps, boundary: str = OPEN) -> sp.csr_matrix:
    """Tridiagonal one-particle Hamiltonian H1 (N x N, FP64)."""
    eps = np.asarray(eps, dtype=np.float64)
    J = np.asarray(J, dtype=np.float64)
    N = eps.shape[0]
    if J.shape[0] != n_bonds(N, boundary):
        raise ValueError(f"expected {n_bonds(N, boundary)} bonds, got {J.shape[0]}")
    if boundary == PERIODIC and N < 3:
        raise ValueError("periodic chain needs N >= 3")
    rows, cols, vals = list(range(N)), list(range(N)), list(eps)
    for i, Ji in enumerate(J):
        a, b = i, (i + 1) % N
        rows += [a, b]
        cols += [b, a]
        vals += [Ji, Ji]
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def pair_distance(xa: np.ndarray, xb: np.ndarray, N: int, boundary: str) -> np.ndarray:
    d = np.abs(xa - xb)
    if boundary == PERIODIC:
        d = np.minimum(d, N - d)
    return d


def interaction_diagonal(states: np.ndarray, N: int, U: float,
                         interaction: str = ONSITE, boundary: str = OPEN) -> np.ndarray:
    """V(x) for each basis tuple (FP64)."""
    m = states.shape[1]
    count = np.zeros(states.shape[0], dtype=np.float64)
    for a in range(m):
        for b in range(a + 1, m):
            d = pair_distance(states[:, a], states[:, b], N, boundary)
            if interaction == ONSITE:
                count += (d == 0)
            elif interaction == NEAREST:
                count += (d == 1)
            else:
                raise ValueError(f"unknown interaction {interaction!r}")
    return U * count


def full_hamiltonian(N: int, m: int, J, eps, U: float, boundary: str = OPEN,
                     interaction: str = ONSITE) -> sp.csr_matrix:
    """H on the full N^m grid (distinguishable particles)."""
    H1 = single_particle(J, eps, boundary)
    eye = sp.identity(N, format="csr", dtype=np.float64)
    H = sp.csr_matrix((N ** m, N ** m), dtype=np.float64)
    for a in range(m):
        term = None
        for b in range(m):
            factor = H1 if b == a else eye
            term = factor if term is None else sp.kron(term, factor, format="csr")
        H = H + term
    V = interaction_diagonal(basis_states(N, m, DISTINGUISHABLE), N, U, interaction, boundary)
    return (H + sp.diags(V, format="csr")).tocsr()


def hamiltonian(N: int, m: int, J, eps, U: float, statistics: str = DISTINGUISHABLE,
                boundary: str = OPEN, interaction: str = ONSITE) -> sp.csr_matrix:
    """H in the basis of ``basis.basis_states(N, m, statistics)``."""
    H = full_hamiltonian(N, m, J, eps, U, boundary, interaction)
    if statistics == DISTINGUISHABLE:
        return H
    if statistics == BOSON:
        S = symmetrizer(N, m)
        return (S.T @ H @ S).tocsr()
    if statistics == FERMION:
        A = antisymmetrizer(N, m)
        return (A.T @ H @ A).tocsr()
    raise ValueError(f"unknown statistics {statistics!r}")


def bond_operator(N: int, m: int, bond: int, statistics: str = DISTINGUISHABLE,
                  boundary: str = OPEN) -> sp.csr_matrix:
    """dH/dJ_bond: the hopping operator of one bond for every particle."""
    J = np.zeros(n_bonds(N, boundary))
    J[bond] = 1.0
    return hamiltonian(N, m, J, np.zeros(N), 0.0, statistics, boundary)


def site_operator(N: int, m: int, site: int, statistics: str = DISTINGUISHABLE,
                  boundary: str = OPEN) -> sp.csr_matrix:
    """dH/deps_site: the occupation operator of one node."""
    eps = np.zeros(N)
    eps[site] = 1.0
    return hamiltonian(N, m, np.zeros(n_bonds(N, boundary)), eps, 0.0, statistics, boundary)
