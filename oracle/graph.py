"""One particle on a general graph (Sec. 2) for checking the library.  Test
infrastructure only: nothing in the product path imports this module.

Sec. 2 lets each node couple to its own set of neighbours; a q-dimensional
regular lattice with nearest-neighbour coupling along each axis is one such
graph.  For one particle H is then the n x n matrix of Eq. (1) with
H[a, a] = eps_a on the diagonal and H[a, b] = H[b, a] = J_e for each bond
e = (a, b) (equal rates both ways, Sec. 2.2), zero elsewhere.  The
evolution itself is ``propagate.evolve_taylor`` on this H.

Pins in tests/test_oracle_pins.py: the clean lattice spectra against the
closed forms (sums of 2 cos(pi k / (N + 1)) over the axes, open; sums of
2 cos(2 pi k / N), periodic), node degrees, symmetry, the two-node closed
form; for two particles, the non-interacting spectra (sums of one-particle
eigenvalues: ordered pairs, pairs i <= j for bosons, i < j for fermions)
and, on a chain, the pinned many-particle chain Hamiltonian.
"""

from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def lattice_bonds(shape, periodic=False):
    """Bonds of the lattice with sides ``shape``: node (c_1, ..., c_q) is
    numbered row-major; each node is joined to the next node along every
    axis (and, on a periodic axis longer than 2, the last to the first).
    Returned as a sorted list of (a, b) with a < b."""
    shape = tuple(int(s) for s in shape)
    strides = [int(np.prod(shape[i + 1:])) for i in range(len(shape))]
    bonds = set()
    for c in itertools.product(*[range(s) for s in shape]):
        a = sum(ci * st for ci, st in zip(c, strides))
        for ax, s in enumerate(shape):
            nxt = c[ax] + 1
            if nxt == s:
                if not (periodic and s > 2):
                    continue
                nxt = 0
            b = a + (nxt - c[ax]) * strides[ax]
            bonds.add((min(a, b), max(a, b)))
    return sorted(bonds)


def hamiltonian(n, bonds, J, eps):
    """H of one realisation: eps on the diagonal, J[e] on both entries of
    bond e."""
    H = sp.lil_matrix((n, n), dtype=np.float64)
    for a in range(n):
        H[a, a] = eps[a]
    for (a, b), j in zip(bonds, J):
        H[a, b] += j
        H[b, a] += j
    return H.tocsr()


FERMION = "fermion"


def antisymmetrizer(n):
    """Isometry from the two-fermion states to the n^2 grid: column k, for
    the k-th pair a < b in lexicographic order, is (|a b> - |b a>) / sqrt 2
    (row-major grid index a * n + b)."""
    A, B = np.triu_indices(n, 1)
    k = np.arange(len(A))
    rows = np.concatenate([A * n + B, B * n + A])
    vals = np.concatenate([np.full(len(A), 1 / np.sqrt(2)), np.full(len(A), -1 / np.sqrt(2))])
    return sp.csr_matrix((vals, (rows, np.concatenate([k, k]))), shape=(n * n, len(A)))


def pair_hamiltonian(n, bonds, J, eps, U, statistics):
    """Two particles on the graph (Eq. 1 with m = 2): the one-particle H
    acting on either particle, H1 x 1 + 1 x H1, plus U on the states with
    both particles on one node (on-site interaction).  Distinguishable:
    the n^2 grid in row-major order; bosons: S^T H S with the symmetrising
    isometry of ``basis.symmetrizer`` (sorted pairs, lexicographic);
    fermions: the same with the antisymmetrising isometry (pairs a < b,
    lexicographic), where U drops out since no node holds two."""
    from .basis import BOSON, symmetrizer
    H1 = hamiltonian(n, bonds, J, eps)
    one = sp.identity(n, format="csr")
    H = sp.kron(H1, one) + sp.kron(one, H1)
    double = np.array([float(a == b) for a in range(n) for b in range(n)])
    H = (H + sp.diags(U * double)).tocsr()
    if statistics == BOSON:
        S = symmetrizer(n, 2)
        H = (S.T @ H @ S).tocsr()
    elif statistics == FERMION:
        S = antisymmetrizer(n)
        H = (S.T @ H @ S).tocsr()
    return H
