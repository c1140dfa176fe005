"""Many-particle basis of m particles on an N-site chain (oracle, FP64 CPU).

Sec. 2 of the paper: the walk of m particles on N nodes lives in an
N^m-dimensional space, one amplitude per tuple of occupied nodes.

* Distinguishable particles: every tuple (x_1, ..., x_m), 0 <= x_a < N,
  enumerated lexicographically with x_m running fastest, so that the index of
  a tuple is sum_a x_a N^(m-a) (row-major over the m-dimensional grid).
* Bosons: the exchange-symmetric sector.  One basis state per sorted tuple
  x_1 <= ... <= x_m (lexicographic order), namely the normalised symmetric
  combination of all distinct permutations of that tuple.  ``symmetrizer``
  returns the explicit isometry S from this sector into the full N^m space.
* Fermions: the exchange-antisymmetric sector.  One basis state per
  strictly increasing tuple x_1 < ... < x_m (lexicographic order), the
  normalised combination of all permutations P of the tuple with the sign
  of P; ``antisymmetrizer`` returns the isometry into the full space.

Test infrastructure only; see the package docstring.
"""

from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

DISTINGUISHABLE = "distinguishable"
BOSON = "boson"
FERMION = "fermion"


def basis_states(N: int, m: int, statistics: str = DISTINGUISHABLE) -> np.ndarray:
    """Return the basis tuples as an int64 array of shape (D, m)."""
    if N < 1 or m < 1:
        raise ValueError("need N >= 1 and m >= 1")
    if statistics == DISTINGUISHABLE:
        grids = np.meshgrid(*([np.arange(N)] * m), indexing="ij")
        return np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.int64)
    if statistics == BOSON:
        rows = list(itertools.combinations_with_replacement(range(N), m))
        return np.asarray(rows, dtype=np.int64).reshape(len(rows), m)
    if statistics == FERMION:
        rows = list(itertools.combinations(range(N), m))
        return np.asarray(rows, dtype=np.int64).reshape(len(rows), m)
    raise ValueError(f"unknown statistics {statistics!r}")


def dimension(N: int, m: int, statistics: str = DISTINGUISHABLE) -> int:
    if statistics == DISTINGUISHABLE:
        return N ** m
    if statistics == BOSON:
        return math.comb(N + m - 1, m)
    if statistics == FERMION:
        return math.comb(N, m)
    raise ValueError(f"unknown statistics {statistics!r}")


def full_index(tuples: np.ndarray, N: int) -> np.ndarray:
    """Row-major index of each tuple in the full N^m grid."""
    tuples = np.asarray(tuples, dtype=np.int64)
    idx = np.zeros(tuples.shape[0], dtype=np.int64)
    for a in range(tuples.shape[1]):
        idx = idx * N + tuples[:, a]
    return idx


def symmetrizer(N: int, m: int) -> sp.csr_matrix:
    """Isometry S (N^m x D_boson) whose column k is the normalised symmetric
    state built from the k-th sorted tuple.

    For a sorted tuple with distinct permutations P_1..P_p the column holds
    1/sqrt(p) at each permuted tuple; S^T S is the identity.
    """
    sym = basis_states(N, m, BOSON)
    rows, cols, vals = [], [], []
    for k, t in enumerate(sym):
        perms = sorted(set(itertools.permutations(tuple(int(v) for v in t))))
        w = 1.0 / math.sqrt(len(perms))
        for p in perms:
            rows.append(int(full_index(np.asarray([p]), N)[0]))
            cols.append(k)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N ** m, sym.shape[0]))


def permutation_sign(seq) -> int:
    """Sign of the permutation that sorts a sequence of distinct values
    (by counting inversions)."""
    seq = list(seq)
    inv = sum(1 for i in range(len(seq)) for j in range(i + 1, len(seq)) if seq[i] > seq[j])
    return -1 if inv % 2 else 1


def antisymmetrizer(N: int, m: int) -> sp.csr_matrix:
    """Isometry A (N^m x D_fermion) whose column k is the normalised
    antisymmetric state of the k-th increasing tuple t: 1/sqrt(m!) times the
    sign of P at each permuted tuple P(t); A^T A is the identity."""
    fer = basis_states(N, m, FERMION)
    rows, cols, vals = [], [], []
    w = 1.0 / math.sqrt(math.factorial(m))
    for k, t in enumerate(fer):
        for p in itertools.permutations(tuple(int(v) for v in t)):
            rows.append(int(full_index(np.asarray([p]), N)[0]))
            cols.append(k)
            vals.append(w * permutation_sign(p))
    return sp.csr_matrix((vals, (rows, cols)), shape=(N ** m, fer.shape[0]))


def product_state(N: int, sites, statistics: str = DISTINGUISHABLE) -> np.ndarray:
    """Initial state with particle a on node sites[a] (complex128, in the
    basis of ``basis_states``).  For bosons the normalised symmetric state
    of that occupation; for fermions the normalised antisymmetric state
    (the Slater determinant of the occupied nodes, particle a on sites[a]),
    whose coefficient on the sorted tuple is the sign of the permutation
    that sorts ``sites``."""
    sites = [int(s) for s in sites]
    m = len(sites)
    if any(s < 0 or s >= N for s in sites):
        raise ValueError("start site out of range")
    D = dimension(N, m, statistics)
    psi = np.zeros(D, dtype=np.complex128)
    if statistics == DISTINGUISHABLE:
        psi[int(full_index(np.asarray([sites]), N)[0])] = 1.0
        return psi
    if statistics == FERMION and len(set(sites)) != m:
        raise ValueError("two fermions on one node")
    key = tuple(sorted(sites))
    states = basis_states(N, m, statistics)
    hit = np.nonzero((states == np.asarray(key)).all(axis=1))[0]
    psi[int(hit[0])] = float(permutation_sign(sites)) if statistics == FERMION else 1.0
    return psi
