"""Observables from the diagonal of the ensemble-averaged density matrix.

Eq. (2) and the post-processing stage of Algs. 1-3: each realisation gives
rho_r = |psi_r><psi_r| and the ensemble average is <rho> = (1/R) sum_r rho_r.
The paper leaves the post-processed observables unnamed; the ones built here
depend only on the diagonal of <rho> in the occupation basis, i.e. on the
probabilities p_r(x) = |psi_r(x)|^2 of the basis tuples x:

* occupation   n(i)    = sum_x p(x) * #{a : x_a = i}           (sums to m)
* pair corr.   G(i, j) = sum_x p(x) * #{a != b : x_a = i, x_b = j}
  (the normal-ordered <n_i n_j> - delta_ij <n_i>; sum_j G(i,j) = (m-1) n(i))
* marginal     P_a(i)  = sum_x p(x) [x_a = i]  (distinguishable particles)

Both operators are symmetric under particle exchange, so they are diagonal
in the symmetric (boson) basis as well and the same formulas apply there
with the sorted tuples.

Test infrastructure only; see the package docstring.
"""

from __future__ import annotations

import math

import numpy as np


def probabilities(psi) -> np.ndarray:
    psi = np.asarray(psi, dtype=np.complex128)
    return psi.real ** 2 + psi.imag ** 2


def occupation(psi, states: np.ndarray, N: int) -> np.ndarray:
    p = probabilities(psi)
    out = np.zeros(N, dtype=np.float64)
    for a in range(states.shape[1]):
        out += np.bincount(states[:, a], weights=p, minlength=N)
    return out


def marginal(psi, states: np.ndarray, N: int, particle: int) -> np.ndarray:
    p = probabilities(psi)
    return np.bincount(states[:, particle], weights=p, minlength=N)


def pair_correlation(psi, states: np.ndarray, N: int) -> np.ndarray:
    p = probabilities(psi)
    m = states.shape[1]
    out = np.zeros((N, N), dtype=np.float64)
    for a in range(m):
        for b in range(m):
            if a == b:
                continue
            np.add.at(out, (states[:, a], states[:, b]), p)
    return out


def norm2(psi) -> float:
    return float(np.sum(probabilities(psi)))


def ensemble_mean(per_realization) -> np.ndarray:
    """(1/R) sum_r values_r, summed in realisation order in FP64."""
    arr = np.asarray(per_realization, dtype=np.float64)
    acc = np.zeros(arr.shape[1:], dtype=np.float64)
    for r in range(arr.shape[0]):
        acc = acc + arr[r]
    return acc / arr.shape[0]


def exact_mean(values) -> float:
    """Correctly rounded mean of a 1-D list (math.fsum), for checks."""
    values = [float(v) for v in values]
    return math.fsum(values) / len(values)


def density_matrix(states) -> np.ndarray:
    """<rho> = (1/R) sum_r |psi_r><psi_r| (Eq. 2), the full matrix, from the
    realisations' coefficient vectors in one basis (rows of `states`)."""
    states = [np.asarray(s, dtype=np.complex128) for s in states]
    rho = np.zeros((states[0].size, states[0].size), dtype=np.complex128)
    for psi in states:
        rho += np.outer(psi, psi.conj())
    return rho / len(states)
