"""Seeded synthetic workloads for noisy many-particle quantum walks.

This module only draws inputs: lattice sizes, static noise on the hoppings
and on-site energies, interaction strengths and start sites.  It holds none
of the method's arithmetic (no Hamiltonian, no propagation, no
observables), and it is the one module that both the FP64 oracle tests and
the GPU path consume, so that the two sides see identical parameters.

Noise model (Sec. 2, Eq. 1 of the paper: deterministic plus stochastic
entries; static in time here): realisation r has
    J^r_i   = Jbar_i   + dJ^r_i      (bond i between nodes i and i+1)
    eps^r_i = epsbar_i + deps^r_i
    U^r     = Ubar     + dU^r
with the draws independent across realisations.  Each realisation draws
from its own counter-based stream, numpy's Philox keyed by (seed, r), in
the order: bonds, then sites, then U, so any subset of realisations can be
regenerated on its own.

Workloads follow the paper's benchmark setting (one-dimensional chains,
two particles, nearest-neighbour hopping, noisy tunnelling, R ~ 1000
realisations, Sec. 4) and extend it to bosons, uneven batches and three
particles.
"""

from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

DIST_NONE = "none"
DIST_UNIFORM = "uniform"   # U[a, b]
DIST_NORMAL = "normal"     # N(a, b^2)


@dataclasses.dataclass(frozen=True)
class Noise:
    dist: str = DIST_NONE
    a: float = 0.0
    b: float = 0.0

    def draw(self, rng: np.random.Generator, n: int) -> np.ndarray:
        if self.dist == DIST_NONE:
            return np.zeros(n)
        if self.dist == DIST_UNIFORM:
            return rng.uniform(self.a, self.b, size=n)
        if self.dist == DIST_NORMAL:
            return rng.normal(self.a, self.b, size=n)
        raise ValueError(self.dist)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    m: int
    statistics: str                 # "distinguishable" | "boson"
    R: int
    N: int = 0                      # uniform lattice size, or 0 with N_choices
    N_choices: Optional[Sequence[int]] = None   # uneven batch: N_r ~ U{choices}
    boundary: str = "open"
    interaction: str = "onsite"     # "onsite" | "nearest"
    Jbar: float = 1.0
    epsbar: float = 0.0
    Ubar: float = 0.0
    J_noise: Noise = Noise()
    eps_noise: Noise = Noise()
    U_noise: Noise = Noise()
    dt: float = 0.01
    n_steps: int = 100
    output_every: int = 10
    tol: float = 1e-14
    dtype: str = "c128"
    start: Optional[Sequence[int]] = None   # None: centred sites
    seed: int = 0

    def lattice_sizes(self) -> np.ndarray:
        if self.N_choices is None:
            return np.full(self.R, self.N, dtype=np.int64)
        rng = np.random.Generator(np.random.Philox(key=self.seed + (0xC0FFEE << 64)))
        idx = rng.integers(0, len(self.N_choices), size=self.R)
        return np.asarray(self.N_choices, dtype=np.int64)[idx]

    def n_bonds(self, N: int) -> int:
        return N - 1 if self.boundary == "open" else N

    def start_sites(self, N: int) -> list:
        if self.start is not None:
            return [int(s) for s in self.start]
        if self.m == 1:
            return [N // 2]
        if self.m == 2:
            return [N // 2 - 1, N // 2]
        return [N // 2 - 1, N // 2, N // 2 + 1]

    def realization(self, r: int, N: Optional[int] = None):
        """(J[n_bonds], eps[N], U) of realisation r, FP64."""
        if N is None:
            N = int(self.lattice_sizes()[r])
        rng = np.random.Generator(np.random.Philox(key=self.seed + (int(r) << 64)))
        J = self.Jbar + self.J_noise.draw(rng, self.n_bonds(N))
        eps = self.epsbar + self.eps_noise.draw(rng, N)
        U = self.Ubar + float(self.U_noise.draw(rng, 1)[0])
        return J, eps, U

    def noise_only(self, r: int, N: Optional[int] = None):
        """The draws alone (dJ, deps, U) of realisation r."""
        J, eps, U = self.realization(r, N)
        return J - self.Jbar, eps - self.epsbar, U

    def all_realizations(self, subset: Optional[Sequence[int]] = None):
        sizes = self.lattice_sizes()
        rs = range(self.R) if subset is None else subset
        return [(int(sizes[r]),) + self.realization(r, int(sizes[r])) for r in rs]


def C1() -> Workload:
    """Two distinguishable walkers, N=16 open chain, J_i = 1 + U[-0.1,0.1],
    8 realisations, dt=0.01 to t=5, output every 0.1, complex128."""
    return Workload("C1_m2_dist_N16", m=2, statistics="distinguishable", R=8, N=16,
                    J_noise=Noise(DIST_UNIFORM, -0.1, 0.1), dt=0.01, n_steps=500,
                    output_every=10, tol=1e-14, dtype="c128", start=(7, 8))


def C2(dtype: str = "c128") -> Workload:
    """Two bosons, N=128 open chain, on-site U=2, J~N(1,0.2^2),
    eps~U[-0.5,0.5], 1000 realisations, dt=0.05 to t=50."""
    return Workload("C2_m2_boson_N128", m=2, statistics="boson", R=1000, N=128, Ubar=2.0,
                    J_noise=Noise(DIST_NORMAL, 0.0, 0.2),
                    eps_noise=Noise(DIST_UNIFORM, -0.5, 0.5), dt=0.05, n_steps=1000,
                    output_every=20, tol=1e-14 if dtype == "c128" else 1e-7,
                    dtype=dtype, start=(63, 64))


def C3(dtype: str = "c64") -> Workload:
    """Uneven batch: 4096 realisations of two distinguishable walkers on
    open chains with N_r ~ U{64, 96, ..., 1024}, U_r ~ U[0,4], J~N(1,0.1^2),
    eps = 0, dt=0.05, 200 steps, output every 50."""
    return Workload("C3_m2_uneven_N64-1024", m=2, statistics="distinguishable", R=4096,
                    N_choices=tuple(range(64, 1025, 32)),
                    U_noise=Noise(DIST_UNIFORM, 0.0, 4.0),
                    J_noise=Noise(DIST_NORMAL, 0.0, 0.1), dt=0.05, n_steps=200,
                    output_every=50, tol=1e-7 if dtype == "c64" else 1e-14, dtype=dtype)


def C4(dtype: str = "c128", start=(191, 192)) -> Workload:
    """Gradient workload: two bosons on N=256, U=1, J = 1 + N(0,0.1^2),
    eps = U[-0.5,0.5], 512 realisations, dt=0.05, 400 steps (t=20)."""
    return Workload("C4_m2_boson_N256_adjoint", m=2, statistics="boson", R=512, N=256,
                    Ubar=1.0, J_noise=Noise(DIST_NORMAL, 0.0, 0.1),
                    eps_noise=Noise(DIST_UNIFORM, -0.5, 0.5), dt=0.05, n_steps=400,
                    output_every=400, tol=1e-14 if dtype == "c128" else 1e-7,
                    dtype=dtype, start=start)


def C5() -> Workload:
    """Three distinguishable walkers on N=256, nearest-neighbour U=1,
    eps~U[-1,1], J=1, 64 realisations, dt=0.02 to t=10, complex64."""
    return Workload("C5_m3_dist_N256", m=3, statistics="distinguishable", R=64, N=256,
                    interaction="nearest", Ubar=1.0,
                    eps_noise=Noise(DIST_UNIFORM, -1.0, 1.0), dt=0.02, n_steps=500,
                    output_every=50, tol=1e-7, dtype="c64", start=(127, 128, 129))


def scaled(w: Workload, **changes) -> Workload:
    """A copy of a workload with some fields replaced (smaller parity cases)."""
    return dataclasses.replace(w, **changes)
