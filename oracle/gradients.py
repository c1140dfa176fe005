"""Reference derivatives of an ensemble-averaged diagonal observable (oracle).

The paper evolves R independent realisations and averages rho (Eq. 2);
it does not differentiate.  This module is the FP64 reference for the
derivative extension: realisation r has hoppings J^r = Jbar + dJ^r and
on-site energies eps^r = epsbar + deps^r (additive static noise, fixed
draws), interaction U^r, start state psi_0, and the loss

    L(Jbar, epsbar) = (1/R) sum_r <psi_r(T)| W |psi_r(T)>,

with W diagonal in the occupation basis:
    one-body  w(x) = sum_a g[x_a]
    product   w(x) = prod_a h[x_a]
(the product form with h the indicator of a block of nodes is the
probability that all particles sit in that block).

Two independent routes are given:

* ``fd_gradient``  -- central finite differences of any loss function,
  e.g. ``loss_taylor`` (the truncated-Taylor map of Alg. 3 with a fixed
  number of terms per step) or ``loss_exact`` (exact evolution).
* ``ed_gradient``  -- the exact derivative of the exact evolution
  psi(T) = exp(-i H T) psi_0, from the eigen-decomposition H = V diag(E) V^T
  and the Daleckii-Krein formula for the Frechet derivative of a matrix
  function: d exp(-i H T)[X] = V (F o (V^T X V)) V^T with
  F_ab = (exp(-i T E_a) - exp(-i T E_b)) / (E_a - E_b) and
  F_aa = -i T exp(-i T E_a), written in the numerically stable form
  F_ab = -i T exp(-i T (E_a + E_b)/2) sinc(T (E_a - E_b)/2).
  Then dL/dtheta = (1/R) sum_r 2 Re <W psi_r(T)| d exp[dH/dtheta] psi_0>.

Test infrastructure only; see the package docstring.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import basis as B
from . import hamiltonian as Hm
from . import propagate as P

ONE_BODY = "one_body"
PRODUCT = "product"


def diagonal_weights(states: np.ndarray, site_weights, kind: str) -> np.ndarray:
    g = np.asarray(site_weights, dtype=np.float64)
    if kind == ONE_BODY:
        return g[states].sum(axis=1)
    if kind == PRODUCT:
        return g[states].prod(axis=1)
    raise ValueError(f"unknown weight kind {kind!r}")


class Ensemble:
    """Fixed noise draws for R realisations of one lattice."""

    def __init__(self, N, m, statistics, dJ, deps, U, sites, boundary=Hm.OPEN,
                 interaction=Hm.ONSITE):
        self.N, self.m, self.statistics = N, m, statistics
        self.dJ = np.atleast_2d(np.asarray(dJ, dtype=np.float64))
        self.deps = np.atleast_2d(np.asarray(deps, dtype=np.float64))
        self.U = np.asarray(U, dtype=np.float64).reshape(-1)
        self.R = self.dJ.shape[0]
        self.boundary, self.interaction = boundary, interaction
        self.states = B.basis_states(N, m, statistics)
        self.psi0 = B.product_state(N, sites, statistics)

    def hamiltonian(self, r, Jbar, epsbar):
        return Hm.hamiltonian(self.N, self.m, Jbar + self.dJ[r], epsbar + self.deps[r],
                              float(self.U[r]), self.statistics, self.boundary,
                              self.interaction)


def loss_taylor(ens: Ensemble, Jbar, epsbar, weights, dt, n_steps, order) -> float:
    total = 0.0
    for r in range(ens.R):
        H = ens.hamiltonian(r, Jbar, epsbar)
        psi, _, _ = P.evolve_taylor(H, ens.psi0, dt, n_steps, order=order)
        total += float(np.sum(weights * (psi.real ** 2 + psi.imag ** 2)))
    return total / ens.R


def loss_exact(ens: Ensemble, Jbar, epsbar, weights, T) -> float:
    total = 0.0
    for r in range(ens.R):
        psi = P.EDPropagator(ens.hamiltonian(r, Jbar, epsbar)).evolve(ens.psi0, T)
        total += float(np.sum(weights * (psi.real ** 2 + psi.imag ** 2)))
    return total / ens.R


def fd_gradient(loss, Jbar, epsbar, h=1e-5, bonds=None, sites=None):
    """Central differences of loss(Jbar, epsbar) with step h*max(1,|theta|)."""
    Jbar = np.asarray(Jbar, dtype=np.float64)
    epsbar = np.asarray(epsbar, dtype=np.float64)
    bonds = range(Jbar.shape[0]) if bonds is None else bonds
    sites = range(epsbar.shape[0]) if sites is None else sites
    gJ = np.full(Jbar.shape[0], np.nan)
    ge = np.full(epsbar.shape[0], np.nan)
    for i in bonds:
        step = h * max(1.0, abs(Jbar[i]))
        up, dn = Jbar.copy(), Jbar.copy()
        up[i] += step
        dn[i] -= step
        gJ[i] = (loss(up, epsbar) - loss(dn, epsbar)) / (2 * step)
    for i in sites:
        step = h * max(1.0, abs(epsbar[i]))
        up, dn = epsbar.copy(), epsbar.copy()
        up[i] += step
        dn[i] -= step
        ge[i] = (loss(Jbar, up) - loss(Jbar, dn)) / (2 * step)
    return gJ, ge


def fd_directional(loss, Jbar, epsbar, vJ, veps, h=1e-5) -> float:
    """Central difference of loss along the direction (vJ, veps)."""
    Jbar = np.asarray(Jbar, dtype=np.float64)
    epsbar = np.asarray(epsbar, dtype=np.float64)
    return (loss(Jbar + h * vJ, epsbar + h * veps)
            - loss(Jbar - h * vJ, epsbar - h * veps)) / (2 * h)


def _frechet_kernel(E, T):
    a = E[:, None]
    b = E[None, :]
    return -1j * T * np.exp(-0.5j * T * (a + b)) * np.sinc(T * (a - b) / (2 * np.pi))


def ed_gradient(ens: Ensemble, Jbar, epsbar, weights, T):
    """Exact dL/dJbar and dL/depsbar of the exact evolution (Daleckii-Krein)."""
    N, m = ens.N, ens.m
    nb = Hm.n_bonds(N, ens.boundary)
    bond_ops = [Hm.bond_operator(N, m, i, ens.statistics, ens.boundary).tocoo()
                for i in range(nb)]
    site_ops = [Hm.site_operator(N, m, i, ens.statistics, ens.boundary).tocoo()
                for i in range(N)]
    gJ = np.zeros(nb)
    ge = np.zeros(N)
    for r in range(ens.R):
        H = ens.hamiltonian(r, np.asarray(Jbar, float), np.asarray(epsbar, float)).toarray()
        E, V = sla.eigh(H)
        a = V.T @ ens.psi0
        psiT = V @ (np.exp(-1j * E * T) * a)
        bvec = V.T @ (weights * psiT)
        M = np.conj(bvec)[:, None] * _frechet_kernel(E, T) * a[None, :]
        G = V @ M @ V.T
        for i, op in enumerate(bond_ops):
            gJ[i] += 2.0 * np.real(np.sum(op.data * G[op.row, op.col]))
        for i, op in enumerate(site_ops):
            ge[i] += 2.0 * np.real(np.sum(op.data * G[op.row, op.col]))
    return gJ / ens.R, ge / ens.R
