"""Switching (telegraph) hopping noise, Eq. 1 with time-dependent stochastic
terms, for checking the library.  Test infrastructure only: nothing in the
product path imports this module.

Each bond i of realisation r carries xi_i(t) = +-a, flipping sign at the
events of a Poisson process of rate g; per time step of length dt the bond
flips at the start of the step with probability p = 1 - exp(-g dt), and
J_i = Jbar_i + xi_i holds during the step.  The draws follow the library's
documented mapping (include/ctqw.h, ctqw_set_telegraph): Philox4x32-10 from
``oracle.noise`` with counter (i, 4 (s + 1), r mod 2^32, r div 2^32) and key
(seed mod 2^32 XOR 0x54454C45, seed div 2^32); u = 53-bit fraction of
(w0, w1); s = -1 is the initial sign (+ if u < 1/2), s >= 0 the flip test
of step s (flip if u < p).
"""

from __future__ import annotations

import math

import numpy as np

from . import noise as Nz
from . import propagate as P

MASK32 = 0xFFFFFFFF
TELE_KEY = 0x54454C45


def _u(seed: int, r: int, i: int, s: int) -> float:
    w = Nz.philox4x32([i, 4 * (s + 1), r & MASK32, r >> 32], [(seed & MASK32) ^ TELE_KEY, seed >> 32])
    return Nz.unit53(w[0], w[1])


def flip_probability(rate: float, dt: float) -> float:
    return -math.expm1(-rate * dt)


def sign_history(seed: int, r: int, n_bonds: int, n_steps: int, p: float) -> np.ndarray:
    """[n_steps, n_bonds] signs in force during steps 0 .. n_steps - 1."""
    sg = np.array([1.0 if _u(seed, r, i, -1) < 0.5 else -1.0 for i in range(n_bonds)])
    out = np.zeros((n_steps, n_bonds))
    for s in range(n_steps):
        for i in range(n_bonds):
            if _u(seed, r, i, s) < p:
                sg[i] = -sg[i]
        out[s] = sg
    return out


def evolve(build_H, Jbar, psi0, dt: float, n_steps: int, order: int, amp: float, rate: float, seed: int, r: int):
    """Taylor steps of the given order with J = Jbar + amp * sign(step);
    build_H(J) returns the Hamiltonian for hoppings J."""
    Jbar = np.asarray(Jbar, dtype=np.float64)
    signs = sign_history(seed, r, Jbar.size, n_steps, flip_probability(rate, dt))
    psi = np.asarray(psi0, dtype=np.complex128).copy()
    for s in range(n_steps):
        H = build_H(Jbar + amp * signs[s])
        psi, _, _ = P.taylor_step(H, psi, dt, order)
    return psi
