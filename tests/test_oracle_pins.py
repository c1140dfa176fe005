"""Pins of the FP64 oracle against closed forms, textbook routines, brute
force and invariants.  CPU only.

Each test states which part of the oracle it fixes and which mistake it
would catch.  None of them re-types the oracle's own formula: the checks
come from special functions (Bessel), eigen-solvers of the one-particle
problem (scipy's tridiagonal solver), Pade-based matrix exponentials, an
independent second-quantised construction of H, and symmetries.
"""

import math
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.special as ss

from oracle import basis as B
from oracle import hamiltonian as Hm
from oracle import observables as O
from oracle import propagate as P


def rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- 1 particle

@pytest.mark.parametrize("t", [2.5, 10.0, 20.0])
def test_bessel_closed_form_single_walker(t):
    """Uniform open chain, walker on node s: psi_{s+n}(t) = (-i)^n J_n(2t)
    before the front reaches the ends (pins the hopping sign, the -i of the
    evolution and the tridiagonal layout)."""
    N, s = 256, 128
    H = Hm.hamiltonian(N, 1, np.ones(N - 1), np.zeros(N), 0.0)
    psi0 = B.product_state(N, [s])
    psi = P.EDPropagator(H).evolve(psi0, t)
    n = np.arange(N) - s
    # For negative n, (-i)^n J_n = i^|n| (-1)^|n| J_|n| = (-i)^|n| J_|n|.
    expect = (-1j) ** np.abs(n) * ss.jv(np.abs(n), 2 * t)
    assert np.max(np.abs(psi - expect)) < 1e-12


def test_bessel_reference_values_against_mpmath():
    """scipy's jv is the reference above; cross-check it at high precision."""
    for n, z in [(0, 5.0), (3, 20.0), (17, 40.0), (60, 40.0)]:
        assert abs(ss.jv(n, z) - float(mpmath.besselj(n, z))) < 1e-14


def test_bessel_taylor_and_rk4_routes():
    """Alg. 3 with a tolerance and Alg. 2 with a small step reach the same
    closed form (pins the Taylor recursion Phi_j = -(i dt/j) H Phi_{j-1})."""
    N, s, dt, steps = 128, 64, 0.05, 200
    H = Hm.hamiltonian(N, 1, np.ones(N - 1), np.zeros(N), 0.0)
    psi0 = B.product_state(N, [s])
    n = np.abs(np.arange(N) - s)
    expect = (-1j) ** n * ss.jv(n, 2 * dt * steps)
    psi_t, _, orders = P.evolve_taylor(H, psi0, dt, steps, tol=1e-15)
    assert np.max(np.abs(psi_t - expect)) < 1e-12
    assert min(orders) >= 8
    psi_rk = P.evolve_rk4(H, psi0, 0.01, 1000)
    assert np.max(np.abs(psi_rk - expect)) < 1e-6


def test_periodic_ring_fourier_closed_form():
    """Uniform ring: psi_x(t) = (1/N) sum_k exp(2 pi i k (x-s)/N) exp(-2 i J t cos(2 pi k/N))
    (pins the wrap-around bond)."""
    N, s, J, t = 11, 3, 0.7, 3.3
    H = Hm.hamiltonian(N, 1, np.full(N, J), np.zeros(N), 0.0, boundary=Hm.PERIODIC)
    psi = P.EDPropagator(H).evolve(B.product_state(N, [s]), t)
    k = np.arange(N)
    x = np.arange(N)[:, None]
    expect = (np.exp(2j * np.pi * k * (x - s) / N) * np.exp(-2j * J * t * np.cos(2 * np.pi * k / N))).sum(1) / N
    assert np.max(np.abs(psi - expect)) < 1e-13


# --------------------------------------------------- non-interacting m > 1

def one_particle_orbitals(J, eps, t):
    """exp(-i H1 t) from scipy's tridiagonal eigen-solver (textbook routine)."""
    E, V = sla.eigh_tridiagonal(np.asarray(eps, float), np.asarray(J, float))
    return (V * np.exp(-1j * E * t)) @ V.T


@pytest.mark.parametrize("m", [2, 3])
def test_product_form_distinguishable(m):
    """U = 0: psi(x_1..x_m) = prod_a phi_{s_a}(x_a) with phi = exp(-i H1 t)|s>
    (pins the Kronecker-sum order, and that all particles share one set of
    noisy parameters)."""
    g = rng(1)
    N = 9 if m == 2 else 6
    J = 1 + g.uniform(-0.3, 0.3, N - 1)
    eps = g.uniform(-0.5, 0.5, N)
    sites = [1, 6] if m == 2 else [0, 2, 5]
    t = 1.7
    psi = P.EDPropagator(Hm.hamiltonian(N, m, J, eps, 0.0)).evolve(B.product_state(N, sites), t)
    U1 = one_particle_orbitals(J, eps, t)
    expect = U1[:, sites[0]]
    for s in sites[1:]:
        expect = np.multiply.outer(expect, U1[:, s])
    assert np.max(np.abs(psi - expect.reshape(-1))) < 1e-12


def test_product_form_bosons():
    """U = 0 bosons: the normalised symmetric combination of the orbitals;
    in the symmetric basis c_{x<y} = sqrt(2) psi_full(x,y), c_{xx} = psi_full(x,x)."""
    g = rng(2)
    N = 10
    J = 1 + g.uniform(-0.3, 0.3, N - 1)
    eps = g.uniform(-0.5, 0.5, N)
    a, b, t = 3, 4, 2.3
    U1 = one_particle_orbitals(J, eps, t)
    full = (np.outer(U1[:, a], U1[:, b]) + np.outer(U1[:, b], U1[:, a])) / math.sqrt(2)
    psi = P.EDPropagator(Hm.hamiltonian(N, 2, J, eps, 0.0, B.BOSON)).evolve(
        B.product_state(N, [a, b], B.BOSON), t)
    states = B.basis_states(N, 2, B.BOSON)
    expect = np.where(states[:, 0] < states[:, 1], math.sqrt(2), 1.0) * full[states[:, 0], states[:, 1]]
    assert np.max(np.abs(psi - expect)) < 1e-12


@pytest.mark.parametrize("sites", [(3, 6), (6, 3)])
def test_product_form_fermions(sites):
    """U = 0 fermions: the Slater determinant of the evolved orbitals; in the
    antisymmetric basis c_{x<y} = phi_1(x) phi_2(y) - phi_2(x) phi_1(y) with
    phi_a = exp(-i H1 t)|s_a> (particle a started on sites[a]: swapping the
    start sites flips the sign), and the full-grid state A c is
    antisymmetric under exchange."""
    g = rng(12)
    N = 10
    J = 1 + g.uniform(-0.3, 0.3, N - 1)
    eps = g.uniform(-0.5, 0.5, N)
    t = 2.1
    U1 = one_particle_orbitals(J, eps, t)
    f1, f2 = U1[:, sites[0]], U1[:, sites[1]]
    det = np.outer(f1, f2) - np.outer(f2, f1)
    psi = P.EDPropagator(Hm.hamiltonian(N, 2, J, eps, 0.0, B.FERMION)).evolve(
        B.product_state(N, list(sites), B.FERMION), t)
    states = B.basis_states(N, 2, B.FERMION)
    assert np.max(np.abs(psi - det[states[:, 0], states[:, 1]])) < 1e-12
    full = (B.antisymmetrizer(N, 2) @ psi).reshape(N, N)
    assert np.max(np.abs(full + full.T)) < 1e-15
    assert np.max(np.abs(np.diag(full))) == 0.0
    assert abs(np.linalg.norm(psi) - 1) < 1e-13


def test_two_site_boson_closed_form():
    """N = 2, two bosons: basis (0,0), (0,1), (1,1) and
    H = [[2e0+U, sqrt2 J, 0], [sqrt2 J, e0+e1, sqrt2 J], [0, sqrt2 J, 2e1+U]]."""
    J, e0, e1, U = 0.83, -0.2, 0.35, 1.7
    H = Hm.hamiltonian(2, 2, [J], [e0, e1], U, B.BOSON).toarray()
    r2 = math.sqrt(2)
    expect = np.array([[2 * e0 + U, r2 * J, 0], [r2 * J, e0 + e1, r2 * J], [0, r2 * J, 2 * e1 + U]])
    assert np.max(np.abs(H - expect)) < 1e-15


# ------------------------------------------ brute force, second quantised

def second_quantised(N, m, J, eps, U, statistics, boundary, interaction):
    """H built from occupation numbers, independent of the Kronecker route:
    H = sum_i eps_i n_i + sum_bonds J_b (a+_i a_j + h.c.) + V, where for
    bosons a+_i a_j |..n_i..n_j..> = sqrt((n_i+1) n_j) |..n_i+1..n_j-1..>,
    on-site V = U/2 sum_i n_i (n_i - 1) and nearest V = U sum_bonds n_i n_j."""
    states = [tuple(s) for s in B.basis_states(N, m, statistics)]
    index = {s: k for k, s in enumerate(states)}
    bonds = [(i, i + 1) for i in range(N - 1)]
    if boundary == Hm.PERIODIC:
        bonds.append((N - 1, 0))
    H = np.zeros((len(states), len(states)))
    for k, s in enumerate(states):
        occ = np.bincount(s, minlength=N)
        diag = float(np.dot(eps, occ))
        if interaction == Hm.ONSITE:
            diag += U * 0.5 * float(np.sum(occ * (occ - 1)))
        else:
            diag += U * float(sum(occ[i] * occ[j] for i, j in bonds))
        H[k, k] += diag
        for bi, (i, j) in enumerate(bonds):
            for src, dst in ((i, j), (j, i)):
                if statistics == B.FERMION:
                    # c+_dst c_src on the normal-ordered state c+_x1 ... c+_xm |0>:
                    # Jordan-Wigner sign (-1)^(occupied nodes strictly between)
                    if occ[src] == 0 or occ[dst] == 1:
                        continue
                    lo, hi = min(src, dst), max(src, dst)
                    sign = (-1) ** int(occ[lo + 1:hi].sum())
                    new = occ.copy()
                    new[src] -= 1
                    new[dst] += 1
                    t = tuple(int(v) for v in np.nonzero(new)[0])
                    H[index[t], k] += J[bi] * sign
                    continue
                if statistics == B.DISTINGUISHABLE:
                    for a in range(m):
                        if s[a] == src:
                            t = list(s)
                            t[a] = dst
                            H[index[tuple(t)], k] += J[bi]
                else:
                    if occ[src] == 0:
                        continue
                    new = occ.copy()
                    amp = math.sqrt(occ[src] * (occ[dst] + 1))
                    new[src] -= 1
                    new[dst] += 1
                    t = tuple(sorted(np.repeat(np.arange(N), new)))
                    H[index[t], k] += J[bi] * amp
    return H


@pytest.mark.parametrize("m,statistics,boundary,interaction", [
    (2, B.DISTINGUISHABLE, Hm.OPEN, Hm.ONSITE),
    (3, B.DISTINGUISHABLE, Hm.OPEN, Hm.NEAREST),
    (2, B.BOSON, Hm.OPEN, Hm.ONSITE),
    (3, B.BOSON, Hm.OPEN, Hm.ONSITE),
    (2, B.DISTINGUISHABLE, Hm.PERIODIC, Hm.NEAREST),
    (2, B.BOSON, Hm.PERIODIC, Hm.ONSITE),
    (2, B.FERMION, Hm.OPEN, Hm.NEAREST),
    (2, B.FERMION, Hm.OPEN, Hm.ONSITE),
    (2, B.FERMION, Hm.PERIODIC, Hm.NEAREST),
    (3, B.FERMION, Hm.PERIODIC, Hm.NEAREST),
])
def test_hamiltonian_matches_second_quantised(m, statistics, boundary, interaction):
    g = rng(3)
    N = 4
    nb = Hm.n_bonds(N, boundary)
    J = 1 + g.uniform(-0.4, 0.4, nb)
    eps = g.uniform(-1, 1, N)
    U = 1.3
    H = Hm.hamiltonian(N, m, J, eps, U, statistics, boundary, interaction).toarray()
    Href = second_quantised(N, m, J, eps, U, statistics, boundary, interaction)
    assert np.max(np.abs(H - Href)) < 1e-14


@pytest.mark.parametrize("m,statistics", [(2, B.DISTINGUISHABLE), (3, B.DISTINGUISHABLE), (2, B.BOSON)])
def test_ed_matches_pade_expm(m, statistics):
    """ED (Eq. 4) against scipy's scaling-and-squaring Pade exp(-iHt)."""
    g = rng(4)
    N = 4
    H = Hm.hamiltonian(N, m, 1 + g.uniform(-0.2, 0.2, N - 1), g.uniform(-1, 1, N), 0.9, statistics)
    psi0 = B.product_state(N, list(range(m)), statistics)
    t = 3.1
    a = P.EDPropagator(H).evolve(psi0, t)
    b = sla.expm(-1j * t * H.toarray()) @ psi0
    assert np.max(np.abs(a - b)) < 1e-13


# ------------------------------------------------------ propagator routes

def small_case(seed=5, N=8, statistics=B.DISTINGUISHABLE, U=1.5):
    g = rng(seed)
    J = 1 + g.normal(0, 0.2, N - 1)
    eps = g.uniform(-0.5, 0.5, N)
    H = Hm.hamiltonian(N, 2, J, eps, U, statistics)
    psi0 = B.product_state(N, [N // 2 - 1, N // 2], statistics)
    return H, psi0


@pytest.mark.parametrize("statistics", [B.DISTINGUISHABLE, B.BOSON])
def test_taylor_tolerance_matches_ed(statistics):
    H, psi0 = small_case(statistics=statistics)
    dt, steps = 0.05, 400
    psi, snaps, _ = P.evolve_taylor(H, psi0, dt, steps, tol=1e-14, output_every=100)
    ed = P.EDPropagator(H)
    for k, snap in enumerate(snaps):
        assert np.max(np.abs(snap - ed.evolve(psi0, k * 100 * dt))) < 1e-11


def test_rk4_step_equals_fourth_order_taylor_step():
    """For a linear autonomous system one RK4 step is the degree-4 Taylor
    polynomial of exp(-i H dt) (Sec. 2.3)."""
    H, psi0 = small_case()
    psi = P.EDPropagator(H).evolve(psi0, 0.7)
    a = P.rk4_step(H, psi, 0.08)
    b, j, _ = P.taylor_step(H, psi, 0.08, order=4)
    assert j == 4
    assert np.max(np.abs(a - b)) < 1e-15


def test_rk4_global_error_is_fourth_order():
    H, psi0 = small_case()
    T = 2.0
    exact = P.EDPropagator(H).evolve(psi0, T)
    errs = []
    for steps in (40, 80, 160):
        errs.append(np.max(np.abs(P.evolve_rk4(H, psi0, T / steps, steps) - exact)))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 4.0) < 0.3)
    # RK4 does not conserve the norm exactly (Sec. 2.2).
    psi = P.evolve_rk4(H, psi0, T / 40, 40)
    assert abs(np.linalg.norm(psi) - 1) > 1e-9


def test_fixed_order_truncation_error_scales_as_next_power():
    """Dropping terms j > n costs O(dt^(n+1)) per step: halving dt at fixed n
    cuts the one-step error by about 2^(n+1)."""
    H, psi0 = small_case()
    exact = P.EDPropagator(H)
    for n in (3, 5):
        e1 = np.linalg.norm(P.taylor_step(H, psi0, 0.1, order=n)[0] - exact.evolve(psi0, 0.1))
        e2 = np.linalg.norm(P.taylor_step(H, psi0, 0.05, order=n)[0] - exact.evolve(psi0, 0.05))
        assert abs(math.log2(e1 / e2) - (n + 1)) < 0.35


# ------------------------------------------------------------- invariants

def test_norm_and_energy_conservation():
    H, psi0 = small_case(U=2.0)
    dt = 0.05
    e0 = P.energy(H, psi0)
    psi = psi0
    for _ in range(300):
        psi, _, _ = P.taylor_step(H, psi, dt, tol=1e-15)
    assert abs(np.linalg.norm(psi) - 1) < 1e-12
    assert abs(P.energy(H, psi) - e0) < 1e-11


def test_boson_exchange_symmetry_and_sector_agreement():
    """Distinguishable evolution of a symmetrised start stays symmetric and
    equals the boson-sector evolution mapped back to the full grid."""
    g = rng(6)
    N, U, t = 7, 1.1, 2.9
    J = 1 + g.normal(0, 0.2, N - 1)
    eps = g.uniform(-0.5, 0.5, N)
    a, b = 2, 5
    full0 = np.zeros((N, N), complex)
    full0[a, b] = full0[b, a] = 1 / math.sqrt(2)
    full = P.EDPropagator(Hm.hamiltonian(N, 2, J, eps, U)).evolve(full0.reshape(-1), t).reshape(N, N)
    assert np.max(np.abs(full - full.T)) < 1e-13
    sym = P.EDPropagator(Hm.hamiltonian(N, 2, J, eps, U, B.BOSON)).evolve(
        B.product_state(N, [a, b], B.BOSON), t)
    states = B.basis_states(N, 2, B.BOSON)
    from_full = np.where(states[:, 0] < states[:, 1], math.sqrt(2), 1.0) * full[states[:, 0], states[:, 1]]
    assert np.max(np.abs(sym - from_full)) < 1e-13


def test_time_reversal_of_probabilities():
    """Real H and real psi0: psi(-t) = conj(psi(t)), so |psi(t)|^2 = |psi(-t)|^2."""
    H, psi0 = small_case(U=0.7)
    ed = P.EDPropagator(H)
    p = O.probabilities(ed.evolve(psi0, 1.9))
    q = O.probabilities(ed.evolve(psi0, -1.9))
    assert np.max(np.abs(p - q)) < 1e-14
    assert np.max(np.abs(ed.evolve(psi0, 1.9) - np.conj(ed.evolve(psi0, -1.9)))) < 1e-13


def test_mirror_symmetry_of_occupations():
    """Mirror-symmetric parameters and mirrored starts give mirrored
    occupations (pins bond-index orientation)."""
    g = rng(7)
    N = 9
    half = 1 + g.uniform(-0.3, 0.3, (N - 1) // 2)
    J = np.concatenate([half, half[::-1]])
    eh = g.uniform(-0.5, 0.5, N // 2 + 1)
    eps = np.concatenate([eh, eh[:-1][::-1]])
    H = Hm.hamiltonian(N, 2, J, eps, 1.0)
    st = B.basis_states(N, 2)
    ed = P.EDPropagator(H)
    n1 = O.occupation(ed.evolve(B.product_state(N, [1, 3]), 2.2), st, N)
    n2 = O.occupation(ed.evolve(B.product_state(N, [N - 2, N - 4]), 2.2), st, N)
    assert np.max(np.abs(n1 - n2[::-1])) < 1e-13
    # and a non-symmetric J breaks it (the check has teeth)
    J2 = J.copy()
    J2[0] += 0.3
    ed2 = P.EDPropagator(Hm.hamiltonian(N, 2, J2, eps, 1.0))
    m1 = O.occupation(ed2.evolve(B.product_state(N, [1, 3]), 2.2), st, N)
    m2 = O.occupation(ed2.evolve(B.product_state(N, [N - 2, N - 4]), 2.2), st, N)
    assert np.max(np.abs(m1 - m2[::-1])) > 1e-4


# ------------------------------------------------------------- observables

@pytest.mark.parametrize("m,statistics", [(2, B.DISTINGUISHABLE), (3, B.DISTINGUISHABLE), (2, B.BOSON), (3, B.BOSON)])
def test_occupation_and_pair_correlation_sum_rules(m, statistics):
    g = rng(8)
    N = 5
    states = B.basis_states(N, m, statistics)
    psi = g.normal(size=states.shape[0]) + 1j * g.normal(size=states.shape[0])
    n = O.occupation(psi, states, N)
    G = O.pair_correlation(psi, states, N)
    nrm = O.norm2(psi)
    assert abs(n.sum() - m * nrm) < 1e-12 * nrm
    assert np.max(np.abs(G.sum(axis=1) - (m - 1) * n)) < 1e-12 * nrm
    assert np.max(np.abs(G - G.T)) < 1e-14 * nrm


def test_occupation_brute_force_loops():
    g = rng(9)
    N = 4
    states = B.basis_states(N, 3, B.DISTINGUISHABLE)
    psi = g.normal(size=states.shape[0]) + 1j * g.normal(size=states.shape[0])
    n = np.zeros(N)
    G = np.zeros((N, N))
    for k, s in enumerate(states):
        p = abs(psi[k]) ** 2
        for a in range(3):
            n[s[a]] += p
            for b in range(3):
                if a != b:
                    G[s[a], s[b]] += p
    assert np.allclose(O.occupation(psi, states, N), n, rtol=0, atol=1e-13)
    assert np.allclose(O.pair_correlation(psi, states, N), G, rtol=0, atol=1e-13)
    for a in range(3):
        marg = np.array([sum(abs(psi[k]) ** 2 for k, s in enumerate(states) if s[a] == i) for i in range(N)])
        assert np.allclose(O.marginal(psi, states, N, a), marg, rtol=0, atol=1e-13)


def test_boson_occupation_counts_double_occupancy():
    """|x x>_S holds two particles on node x; |x y>_S one on each."""
    N = 4
    states = B.basis_states(N, 2, B.BOSON)
    for k, s in enumerate(states):
        psi = np.zeros(states.shape[0], complex)
        psi[k] = 1
        n = O.occupation(psi, states, N)
        assert n[s[0]] + (n[s[1]] if s[1] != s[0] else 0) == 2


def test_ensemble_mean_against_fsum():
    g = rng(10)
    vals = g.normal(size=(1000, 3)) * 10.0 ** g.integers(-8, 8, size=(1000, 1))
    mean = O.ensemble_mean(vals)
    for c in range(3):
        assert abs(mean[c] - O.exact_mean(vals[:, c])) <= 1e-14 * np.max(np.abs(vals[:, c]))


# ------------------------------------------------------------ noise draws

def _kat_rows():
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            yield w[:4], w[4:6], w[6:]


def test_philox_known_answer_vectors():
    """Philox4x32-10 against the generator's published known-answer vectors."""
    from oracle import noise
    rows = list(_kat_rows())
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert noise.philox4x32(ctr, key) == out


def test_unit53_and_draw_mappings():
    """The 53-bit fraction spans [0, 1 - 2^-53]; uniform draws land in
    [a, b); Box-Muller normals have the stated mean and variance."""
    from oracle import noise
    assert noise.unit53(0, 0) == 0.0
    assert noise.unit53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert noise.unit53(1 << 31, 0) == 0.5
    u = np.array([noise.draw("uniform", -0.5, 0.25, 7, r, noise.SITE, i) for r in range(40) for i in range(100)])
    assert u.min() >= -0.5 and u.max() < 0.25
    assert abs(u.mean() - (-0.125)) < 4 * 0.75 / math.sqrt(12 * u.size)
    z = np.array([noise.draw("normal", 1.0, 0.2, 3, r, noise.BOND, i) for r in range(50) for i in range(100)])
    n = z.size
    assert abs(z.mean() - 1.0) < 4 * 0.2 / math.sqrt(n)
    assert abs(z.var() / 0.04 - 1.0) < 4 * math.sqrt(2.0 / n)
    assert noise.draw("none", 1.0, 2.0, 0, 0, 0, 0) == 0.0
    # distinct counters and keys give distinct blocks
    assert noise.philox4x32([0, 0, 0, 0], [0, 0]) != noise.philox4x32([1, 0, 0, 0], [0, 0])
    assert noise.philox4x32([0, 0, 0, 0], [0, 0]) != noise.philox4x32([0, 0, 0, 0], [1, 0])


def test_density_matrix_properties():
    """<rho> from the oracle: Hermitian, unit trace, positive semidefinite,
    its diagonal the mean probabilities; a single pure state is a
    projector (rho^2 = rho) and a mixture of orthogonal states is not."""
    from oracle import observables as O
    g = np.random.default_rng(5)
    states = []
    for _ in range(4):
        v = g.standard_normal(12) + 1j * g.standard_normal(12)
        states.append(v / np.linalg.norm(v))
    rho = O.density_matrix(states)
    assert np.allclose(rho, rho.conj().T, atol=1e-15)
    assert abs(np.trace(rho) - 1) < 1e-14
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-14
    assert np.allclose(np.diag(rho).real, np.mean([np.abs(s) ** 2 for s in states], axis=0), atol=1e-15)
    pure = O.density_matrix(states[:1])
    assert np.allclose(pure @ pure, pure, atol=1e-14)
    e = np.eye(12)
    mixed = O.density_matrix([e[0], e[1]])
    assert np.allclose(mixed @ mixed, mixed / 2, atol=1e-15) and not np.allclose(mixed @ mixed, mixed)


def test_density_matrix_orientation():
    """Eq. 2 puts the ket on the left: rho = |psi><psi|, rho[a, b] = psi_a
    conj(psi_b).  The mistake rho^T = conj(rho) passes every check above;
    these fail for it: a known off-diagonal phase (psi = (1, i)/sqrt(2)
    gives rho[0, 1] = -i/2), rho |psi> = |psi> for a complex pure state, and
    <phi|rho|phi> = (1/R) sum_r |<phi|psi_r>|^2 for a complex phi."""
    from oracle import observables as O
    rho = O.density_matrix([np.array([1.0, 1j]) / math.sqrt(2.0)])
    assert abs(rho[0, 1] - (-0.5j)) < 1e-15 and abs(rho[1, 0] - 0.5j) < 1e-15
    g = np.random.default_rng(17)
    v = g.standard_normal(9) + 1j * g.standard_normal(9)
    v /= np.linalg.norm(v)
    pure = O.density_matrix([v])
    assert np.max(np.abs(pure @ v - v)) < 1e-15
    assert np.max(np.abs(pure.T @ v - v)) > 1e-2        # the transposed matrix fails
    states = []
    for _ in range(5):
        s = g.standard_normal(9) + 1j * g.standard_normal(9)
        states.append(s / np.linalg.norm(s))
    rho = O.density_matrix(states)
    phi = g.standard_normal(9) + 1j * g.standard_normal(9)
    lhs = np.vdot(phi, rho @ phi)
    rhs = math.fsum(abs(np.vdot(phi, s)) ** 2 for s in states) / len(states)
    assert abs(lhs.imag) < 1e-14 and abs(lhs.real - rhs) < 1e-13
    assert abs(np.vdot(phi, rho.T @ phi).real - rhs) > 1e-3


def _tele_case():
    """Two distinguishable walkers on a 7-node chain (49 states) with noisy
    baselines, for the telegraph pins."""
    g = np.random.default_rng(23)
    N = 7
    Jbar = 1 + 0.1 * g.standard_normal(N - 1)
    eps = g.uniform(-0.3, 0.3, N)
    U = 0.8
    build = lambda J: Hm.hamiltonian(N, 2, J, eps, U)  # noqa: E731
    psi0 = B.product_state(N, [2, 4])
    return N, Jbar, eps, U, build, psi0


def test_telegraph_evolve_reductions():
    """Eq. 1 with switching terms reduces to the static problem: rate 0 is
    the static evolution at Jbar + a s_init (s_init the initial signs), and
    amplitude 0 the static evolution at Jbar, both against
    ``evolve_taylor`` of the same order (pins that evolve applies the
    signs to the hoppings, scaled by a, and nothing else)."""
    from oracle import telegraph as T
    N, Jbar, eps, U, build, psi0 = _tele_case()
    dt, steps, order, a, seed, r = 0.05, 12, 10, 0.3, 9, 2
    s_init = T.sign_history(seed, r, N - 1, 1, 0.0)[0]
    assert set(np.unique(s_init)) == {-1.0, 1.0}            # both signs present: a real test
    got = T.evolve(build, Jbar, psi0, dt, steps, order, a, 0.0, seed, r)
    ref, _, _ = P.evolve_taylor(build(Jbar + a * s_init), psi0, dt, steps, order=order)
    assert np.max(np.abs(got - ref)) < 1e-15
    got0 = T.evolve(build, Jbar, psi0, dt, steps, order, 0.0, 5.0, seed, r)
    ref0, _, _ = P.evolve_taylor(build(Jbar), psi0, dt, steps, order=order)
    assert np.max(np.abs(got0 - ref0)) < 1e-15
    # and a static flip pattern is not a no-op: J differs from Jbar by a
    assert np.max(np.abs(got - ref0)) > 1e-3


def test_telegraph_flip_applies_at_the_start_of_its_step():
    """Flip probability 1 (infinite rate): the signs in force during step 0
    are already the flipped initial signs, then they alternate.  Two steps
    equal one exact step at Jbar - a s_init followed by one at Jbar + a s_init
    (each step against scipy's Pade expm of the dense H, order 30 so the
    Taylor remainder is far below rounding)."""
    from oracle import telegraph as T
    N, Jbar, eps, U, build, psi0 = _tele_case()
    dt, a, seed, r = 0.05, 0.25, 4, 1
    assert T.flip_probability(math.inf, dt) == 1.0
    s_init = T.sign_history(seed, r, N - 1, 1, 0.0)[0]
    got = T.evolve(build, Jbar, psi0, dt, 2, 30, a, math.inf, seed, r)
    H0 = build(Jbar - a * s_init).toarray()
    H1 = build(Jbar + a * s_init).toarray()
    ref = sla.expm(-1j * dt * H1) @ (sla.expm(-1j * dt * H0) @ psi0)
    assert np.max(np.abs(got - ref)) < 1e-14
    # the reading "flip at the end of the step" gives the other order
    wrong = sla.expm(-1j * dt * H0) @ (sla.expm(-1j * dt * H1) @ psi0)
    assert np.max(np.abs(wrong - ref)) > 1e-6


def test_telegraph_sign_process():
    """The switching signs: rate 0 keeps the initial signs, flip
    probability 1 alternates them every step, the initial signs are about
    half positive, and the flip frequency over many steps is within five
    standard deviations of p."""
    from oracle import telegraph as T
    s0 = T.sign_history(7, 3, 64, 5, 0.0)
    assert np.all(s0 == s0[0]) and set(np.unique(s0)) <= {-1.0, 1.0}
    s1 = T.sign_history(7, 3, 64, 4, 1.0)
    assert np.all(s1[1] == -s1[0]) and np.all(s1[2] == s1[0])
    init = T.sign_history(11, 0, 2000, 1, 0.0)[0]
    assert abs(np.mean(init > 0) - 0.5) < 5 * 0.5 / np.sqrt(2000)
    p = T.flip_probability(4.0, 0.05)
    h = T.sign_history(5, 1, 200, 50, p)
    flips = np.sum(h[1:] != h[:-1])
    n = 200 * 49
    assert abs(flips / n - p) < 5 * np.sqrt(p * (1 - p) / n)


# ---------------------------------------------------------------- graphs (Sec. 2)
from oracle import graph as G  # noqa: E402


@pytest.mark.parametrize("shape,periodic", [((5, 7), False), ((3, 4, 5), True), ((6,), False), ((4, 1, 3), False)])
def test_graph_lattice_spectrum_closed_form(shape, periodic):
    """Clean q-dimensional lattice (J = 1, eps = 0): the eigenvalues are the
    sums over the axes of the chain's 2 cos(pi k / (N + 1)), k = 1..N (open)
    or the ring's 2 cos(2 pi k / N) (periodic)."""
    n = int(np.prod(shape))
    bonds = G.lattice_bonds(shape, periodic)
    H = G.hamiltonian(n, bonds, np.ones(len(bonds)), np.zeros(n)).toarray()
    axes = []
    for s in shape:
        if periodic and s > 2:
            axes.append(2 * np.cos(2 * np.pi * np.arange(s) / s))
        elif s == 1:
            axes.append(np.zeros(1))
        else:
            axes.append(2 * np.cos(np.pi * np.arange(1, s + 1) / (s + 1)))
    want = np.zeros(1)
    for ev in axes:
        want = (want[:, None] + ev[None, :]).ravel()
    assert np.allclose(np.linalg.eigvalsh(H), np.sort(want), atol=1e-12)


def test_graph_lattice_degrees_and_bond_count():
    """Open 4 x 6 lattice: (N1 - 1) N2 + N1 (N2 - 1) bonds; interior nodes
    have 4 neighbours, side nodes 3, corners 2; H is symmetric."""
    bonds = G.lattice_bonds((4, 6))
    assert len(bonds) == 3 * 6 + 4 * 5
    deg = np.zeros(24, int)
    for a, b in bonds:
        deg[a] += 1
        deg[b] += 1
    grid = deg.reshape(4, 6)
    assert np.all(grid[1:-1, 1:-1] == 4)
    assert grid[0, 0] == grid[0, -1] == grid[-1, 0] == grid[-1, -1] == 2
    assert np.all(grid[0, 1:-1] == 3) and np.all(grid[1:-1, 0] == 3)
    g = np.random.default_rng(3)
    H = G.hamiltonian(24, bonds, g.standard_normal(len(bonds)), g.standard_normal(24)).toarray()
    assert np.array_equal(H, H.T)


def test_graph_two_node_evolution_closed_form():
    """One bond of coupling J between two nodes, eps = 0: a walker started on
    node 0 has amplitudes (cos Jt, -i sin Jt)."""
    J, t = 0.7, 2.3
    H = G.hamiltonian(2, [(0, 1)], [J], [0.0, 0.0])
    psi, _, _ = P.evolve_taylor(H, np.array([1.0, 0.0]), t / 50, 50, tol=1e-16)
    assert np.allclose(psi, [np.cos(J * t), -1j * np.sin(J * t)], atol=1e-14)


@pytest.mark.parametrize("statistics", [B.DISTINGUISHABLE, B.BOSON])
def test_graph_pair_non_interacting_spectrum(statistics):
    """Two particles, U = 0, on a noisy 3 x 4 lattice: the eigenvalues are
    the sums e_i + e_j of one-particle eigenvalues (all ordered pairs for
    distinguishable particles, i <= j for bosons)."""
    g = np.random.default_rng(8)
    bonds = G.lattice_bonds((3, 4))
    J, eps = 1 + 0.2 * g.standard_normal(len(bonds)), g.uniform(-0.5, 0.5, 12)
    e = np.linalg.eigvalsh(G.hamiltonian(12, bonds, J, eps).toarray())
    if statistics == B.DISTINGUISHABLE:
        want = (e[:, None] + e[None, :]).ravel()
    else:
        i, j = np.triu_indices(12)
        want = e[i] + e[j]
    H = G.pair_hamiltonian(12, bonds, J, eps, 0.0, statistics).toarray()
    assert np.allclose(np.linalg.eigvalsh(H), np.sort(want), atol=1e-12)


@pytest.mark.parametrize("statistics", [B.DISTINGUISHABLE, B.BOSON])
@pytest.mark.parametrize("periodic", [False, True])
def test_graph_pair_on_a_chain_is_the_chain_hamiltonian(statistics, periodic):
    """On the chain graph the two-particle graph H equals the (pinned)
    many-particle chain Hamiltonian with on-site U, open and ring."""
    g = np.random.default_rng(9)
    N = 7
    bonds = G.lattice_bonds((N,), periodic)
    nb = N if periodic else N - 1
    J, eps, U = 1 + 0.2 * g.standard_normal(nb), g.uniform(-0.5, 0.5, N), 1.3
    # the chain module orders bonds i = (i, i + 1), the wrap bond (N - 1, 0) last
    Jb = np.array([J[[k for k, bd in enumerate(bonds) if bd == (min(i, (i + 1) % N), max(i, (i + 1) % N))][0]]
                   for i in range(nb)])
    ref = Hm.hamiltonian(N, 2, Jb, eps, U, statistics, Hm.PERIODIC if periodic else Hm.OPEN, Hm.ONSITE).toarray()
    got = G.pair_hamiltonian(N, bonds, J, eps, U, statistics).toarray()
    assert np.allclose(got, ref, atol=1e-15)


def test_graph_two_fermion_non_interacting_spectrum():
    """Two fermions, noisy 3 x 4 lattice (plaquettes, so exchange signs
    matter): the eigenvalues are e_i + e_j over pairs i < j of distinct
    one-particle eigenvalues, and U has no effect.  Dropping the exchange
    sign of the antisymmetriser (the boson-like isometry on pairs a < b)
    gives another spectrum."""
    g = np.random.default_rng(18)
    bonds = G.lattice_bonds((3, 4))
    J, eps = 1 + 0.2 * g.standard_normal(len(bonds)), g.uniform(-0.5, 0.5, 12)
    e = np.linalg.eigvalsh(G.hamiltonian(12, bonds, J, eps).toarray())
    i, j = np.triu_indices(12, 1)
    want = np.sort(e[i] + e[j])
    for U in (0.0, 2.7):
        H = G.pair_hamiltonian(12, bonds, J, eps, U, G.FERMION).toarray()
        assert H.shape == (66, 66)
        assert np.allclose(np.linalg.eigvalsh(H), want, atol=1e-12)
    S = abs(G.antisymmetrizer(12))
    H1 = G.hamiltonian(12, bonds, J, eps)
    one = sp.identity(12, format="csr")
    wrong = (S.T @ (sp.kron(H1, one) + sp.kron(one, H1)) @ S).toarray()
    assert not np.allclose(np.linalg.eigvalsh(wrong), want, atol=1e-6)


def test_graph_two_fermion_evolution_is_antisymmetric_on_the_grid():
    """Evolving the antisymmetric grid state with the distinguishable pair
    H keeps psi(a, b) = -psi(b, a), and equals the fermion-sector evolution
    mapped back through the antisymmetriser."""
    g = np.random.default_rng(19)
    bonds = G.lattice_bonds((3, 3), periodic=True)
    J, eps = 1 + 0.3 * g.standard_normal(len(bonds)), g.uniform(-1, 1, 9)
    S = G.antisymmetrizer(9)
    c = g.standard_normal(S.shape[1]) + 1j * g.standard_normal(S.shape[1])
    c /= np.linalg.norm(c)
    Hd = G.pair_hamiltonian(9, bonds, J, eps, 0.0, B.DISTINGUISHABLE)
    Hf = G.pair_hamiltonian(9, bonds, J, eps, 0.0, G.FERMION)
    full, _, _ = P.evolve_taylor(Hd, S @ c, 0.02, 40, tol=1e-16)
    sector, _, _ = P.evolve_taylor(Hf, c, 0.02, 40, tol=1e-16)
    grid = full.reshape(9, 9)
    assert np.allclose(grid, -grid.T, atol=1e-13)
    assert np.allclose(full, S @ sector, atol=1e-13)
