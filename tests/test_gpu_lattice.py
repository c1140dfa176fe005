"""GPU parity of one particle on a two-dimensional lattice with every bond
and node carrying its own noisy coupling and energy (Sec. 2, q = 2; Eq. 1),
all Taylor terms of a step in one pass (ctqw_lattice_evolve), against the
oracle's FP64 Taylor map (Eqs. 5-7) of each realisation's H, built by the
oracle's graph Hamiltonian from the same bonds; and against the one-term-
per-pass graph path on the same lattice."""

import numpy as np
import pytest

from oracle import graph as G
from oracle import propagate as P

from _helpers import say

pytestmark = pytest.mark.gpu


def lattice_case(R, Ly, Lx, seed):
    g = np.random.default_rng(seed)
    Jx = 1.0 + 0.1 * g.standard_normal((R, Ly, Lx))
    Jy = 1.0 + 0.1 * g.standard_normal((R, Ly, Lx))
    eps = g.uniform(-0.5, 0.5, (R, Ly, Lx))
    psi = g.standard_normal((R, Ly * Lx)) + 1j * g.standard_normal((R, Ly * Lx))
    psi /= np.linalg.norm(psi, axis=1, keepdims=True)
    return Jx, Jy, eps, psi


def bonds_of(Ly, Lx, px, py, Jx, Jy):
    """Bonds (a, b) of the row-major lattice (node y * Lx + x) with their
    couplings: (x, y)-(x + 1, y) carries Jx[y, x], (x, y)-(x, y + 1) carries
    Jy[y, x]; a periodic axis adds the wrap-around bond."""
    bonds, J = [], []
    for y in range(Ly):
        for x in range(Lx):
            a = y * Lx + x
            if x + 1 < Lx or px:
                bonds.append((a, y * Lx + (x + 1) % Lx))
                J.append(Jx[y, x])
            if y + 1 < Ly or py:
                bonds.append((a, ((y + 1) % Ly) * Lx + x))
                J.append(Jy[y, x])
    return bonds, J


def run_lattice(Jx, Jy, eps, psi0, dt, order, steps, periodic, dtype, norms=False):
    import torch
    from paper_1612_00746_amd import lattice_evolve
    R, Ly, Lx = Jx.shape
    real = torch.float64 if dtype == "c128" else torch.float32
    cplx = torch.complex128 if dtype == "c128" else torch.complex64
    dev = "cuda"
    t = lambda x: torch.tensor(x, dtype=real, device=dev).contiguous()  # noqa: E731
    psi = torch.tensor(psi0.reshape(R, Ly, Lx), dtype=cplx, device=dev).contiguous()
    nrm = torch.zeros((steps, R), dtype=torch.float64, device=dev) if norms else None
    lattice_evolve(t(Jx), t(Jy), t(eps), psi, dt, order, steps, periodic=periodic, norms=nrm)
    torch.cuda.synchronize()
    out = psi.cpu().numpy().reshape(R, Ly * Lx).astype(np.complex128)
    return (out, nrm.cpu().numpy()) if norms else out


@pytest.mark.parametrize("Ly,Lx,px,py,order", [
    (13, 37, False, False, 5),      # one band
    (20, 150, False, False, 8),     # several bands, ragged last band
    (11, 70, True, True, 5),        # ring on both axes
    (9, 130, True, False, 8),       # ring along x, open along y
    (16, 5, False, True, 1),        # narrow, ring along y, one term
])
def test_lattice_c128_against_the_oracle(Ly, Lx, px, py, order):
    R, dt, steps = 3, 0.05, 4
    say(f"case: lattice c128 {Ly}x{Lx} periodic=({px},{py}) order {order}, {steps} steps")
    Jx, Jy, eps, psi0 = lattice_case(R, Ly, Lx, 5)
    got, nrm = run_lattice(Jx, Jy, eps, psi0, dt, order, steps, (px, py), "c128", norms=True)
    worst, worst_n = 0.0, 0.0
    for r in range(R):
        bonds, J = bonds_of(Ly, Lx, px, py, Jx[r], Jy[r])
        H = G.hamiltonian(Ly * Lx, bonds, J, eps[r].ravel())
        ref = psi0[r]
        for k in range(steps):
            ref, _, _ = P.evolve_taylor(H, ref, dt, 1, order=order)
            worst_n = max(worst_n, abs(nrm[k, r] - np.vdot(ref, ref).real))
        worst = max(worst, float(np.max(np.abs(got[r] - ref))))
    say(f"  max |psi - oracle map| = {worst:.2e}, norms {worst_n:.1e}")
    assert worst <= 1e-12 and worst_n <= 1e-12


def test_lattice_c64_against_the_oracle():
    """complex64 with FP32 tables, order 10 (the graph benchmark's), on a
    lattice of several bands: within 1e-6 of the oracle's FP64 map after
    four steps (amplitudes ~0.02; dt-scaled couplings rounded to FP32 and
    one rounding of the state per step)."""
    R, Ly, Lx, dt, order, steps = 3, 24, 140, 0.05, 10, 4
    say(f"case: lattice c64 {Ly}x{Lx} order {order}")
    Jx, Jy, eps, psi0 = lattice_case(R, Ly, Lx, 6)
    got = run_lattice(Jx, Jy, eps, psi0, dt, order, steps, (False, False), "c64")
    worst = 0.0
    for r in range(R):
        bonds, J = bonds_of(Ly, Lx, False, False, Jx[r], Jy[r])
        H = G.hamiltonian(Ly * Lx, bonds, J, eps[r].ravel())
        ref, _, _ = P.evolve_taylor(H, psi0[r], dt, steps, order=order)
        worst = max(worst, float(np.max(np.abs(got[r] - ref))))
    say(f"  max |psi - oracle map| = {worst:.2e}")
    assert worst <= 1e-6


def test_lattice_matches_the_graph_path():
    """The same lattice through ctqw_graph_evolve (one pass per term, ELL
    tables from the bond list) and ctqw_lattice_evolve (all terms in one
    pass): equal to 1e-13 (complex128)."""
    import torch
    from paper_1612_00746_amd import ell_tables, graph_evolve
    R, Ly, Lx, dt, order, steps = 2, 10, 90, 0.05, 7, 3
    say(f"case: lattice vs graph path {Ly}x{Lx}")
    Jx, Jy, eps, psi0 = lattice_case(R, Ly, Lx, 7)
    got = run_lattice(Jx, Jy, eps, psi0, dt, order, steps, (False, False), "c128")
    edges = None
    Jb = []
    for r in range(R):
        bonds, J = bonds_of(Ly, Lx, False, False, Jx[r], Jy[r])
        if r == 0:
            edges = np.array(bonds, dtype=np.int32)
        Jb.append(J)
    nbr, hop = ell_tables(Ly * Lx, edges, np.array(Jb))
    onsite = np.ascontiguousarray(eps.reshape(R, -1))
    dev = "cuda"
    psi = torch.tensor(psi0, dtype=torch.complex128, device=dev).contiguous()
    graph_evolve(torch.tensor(nbr, device=dev), torch.tensor(hop, device=dev), torch.tensor(onsite, device=dev),
                 psi, dt, order, steps)
    torch.cuda.synchronize()
    ref = psi.cpu().numpy()
    diff = float(np.max(np.abs(got - ref)))
    say(f"  max |lattice - graph path| = {diff:.2e}")
    assert diff <= 1e-13
