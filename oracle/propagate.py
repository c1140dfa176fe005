"""FP64 propagators for the time-dependent Schroedinger equation (oracle, CPU).

With hbar = 1, Eq. (2) reads i dpsi/dt = H psi, and for a Hamiltonian that
is static in time the exact solution is psi(t) = exp(-i H t) psi(0).

* ``EDPropagator``  -- exact diagonalisation (Eqs. 3-4, Alg. 1).  One dense
  symmetric eigen-decomposition H = W diag(E) W^T per realisation (H is
  static here), then psi(t) = W (exp(-i E t) * (W^T psi(0))) evaluated
  directly at each requested time t = k dt (a product, not a running sum).
* ``taylor_step`` / ``evolve_taylor`` -- the truncated Taylor series of the
  evolution operator, Eqs. (6)-(7) and Alg. 3: Phi^(0) = psi,
  Phi^(j) = -(i dt / j) H Phi^(j-1), psi(t+dt) = sum_{j<=n} Phi^(j).  The
  paper runs a fixed n; with ``order=None`` the series is cut after the
  first term whose 2-norm is at most ``tol`` times the 2-norm of the partial
  sum (a posteriori), capped at ``max_order``.
* ``rk4_step`` / ``evolve_rk4`` -- classical fourth-order Runge-Kutta on
  dpsi/dt = -i H psi (Sec. 2.2, Alg. 2); the four stages combine with the
  weights 1/6, 1/3, 1/3, 1/6.

Test infrastructure only; see the package docstring.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class EDPropagator:
    """Exact evolution of one static Hamiltonian by diagonalisation."""

    def __init__(self, H):
        Hd = H.toarray() if sp.issparse(H) else np.asarray(H, dtype=np.float64)
        if not np.allclose(Hd, Hd.T, rtol=0, atol=0):
            raise ValueError("H must be real symmetric")
        self.E, self.W = sla.eigh(Hd)

    def evolve(self, psi0, t: float) -> np.ndarray:
        coeff = self.W.T @ np.asarray(psi0, dtype=np.complex128)
        return self.W @ (np.exp(-1j * self.E * t) * coeff)

    def evolve_many(self, psi0, times) -> np.ndarray:
        coeff = self.W.T @ np.asarray(psi0, dtype=np.complex128)
        out = np.empty((len(times), coeff.shape[0]), dtype=np.complex128)
        for k, t in enumerate(times):
            out[k] = self.W @ (np.exp(-1j * self.E * t) * coeff)
        return out


def taylor_step(H, psi, dt: float, order: int | None = None, tol: float = 1e-14,
                max_order: int = 60):
    """One step of Alg. 3.  Returns (psi(t+dt), terms used, ||Phi^(n)||)."""
    phi = np.asarray(psi, dtype=np.complex128).copy()
    out = phi.copy()
    j = 0
    tail = np.linalg.norm(phi)
    while True:
        j += 1
        phi = (-1j * dt / j) * (H @ phi)
        out = out + phi
        tail = np.linalg.norm(phi)
        if order is not None:
            if j >= order:
                break
        else:
            if tail <= tol * np.linalg.norm(out):
                break
            if j >= max_order:
                raise RuntimeError("Taylor series did not reach the tolerance")
    return out, j, tail


def evolve_taylor(H, psi0, dt: float, n_steps: int, order: int | None = None,
                  tol: float = 1e-14, output_every: int | None = None,
                  max_order: int = 60):
    """Repeat ``taylor_step``.  Returns (final psi, snapshots, orders) where
    snapshots holds psi at steps 0, output_every, 2*output_every, ..."""
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    snaps, orders = [], []
    if output_every:
        snaps.append(psi.copy())
    for s in range(1, n_steps + 1):
        psi, j, _ = taylor_step(H, psi, dt, order, tol, max_order)
        orders.append(j)
        if output_every and s % output_every == 0:
            snaps.append(psi.copy())
    return psi, snaps, orders


def rk4_step(H, psi, dt: float) -> np.ndarray:
    """One classical RK4 step of dpsi/dt = -i H psi (Alg. 2)."""
    f = lambda v: -1j * (H @ v)  # noqa: E731
    k1 = f(psi)
    k2 = f(psi + 0.5 * dt * k1)
    k3 = f(psi + 0.5 * dt * k2)
    k4 = f(psi + dt * k3)
    return psi + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def evolve_rk4(H, psi0, dt: float, n_steps: int) -> np.ndarray:
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    for _ in range(n_steps):
        psi = rk4_step(H, psi, dt)
    return psi


def energy(H, psi) -> float:
    """<psi|H|psi> / <psi|psi> (real for real symmetric H)."""
    psi = np.asarray(psi, dtype=np.complex128)
    return float(np.real(np.vdot(psi, H @ psi)) / np.real(np.vdot(psi, psi)))
