"""Pins of the oracle's reference derivatives.  CPU only.

The Daleckii-Krein (eigen-decomposition) gradient and central finite
differences are two independent routes to the same number; a sign error in
the -i of the evolution, a transposed kernel F, a missing factor 2 Re or a
wrong bond orientation in dH/dJ fails the comparison.
"""

import numpy as np
import pytest

from oracle import basis as B
from oracle import gradients as G
from oracle import hamiltonian as Hm


def make_ensemble(statistics, N=6, R=3, seed=11, sites=(2, 3)):
    g = np.random.default_rng(seed)
    dJ = g.normal(0, 0.1, (R, N - 1))
    deps = g.uniform(-0.5, 0.5, (R, N))
    U = g.uniform(0.5, 1.5, R)
    return G.Ensemble(N, 2, statistics, dJ, deps, U, list(sites))


@pytest.mark.parametrize("statistics,kind", [(B.BOSON, G.PRODUCT), (B.DISTINGUISHABLE, G.ONE_BODY)])
def test_ed_gradient_matches_central_differences(statistics, kind):
    ens = make_ensemble(statistics)
    N = ens.N
    site_w = np.zeros(N)
    site_w[N // 2:] = 1.0 if kind == G.PRODUCT else 0.0
    if kind == G.ONE_BODY:
        site_w = np.linspace(-1, 1, N)
    w = G.diagonal_weights(ens.states, site_w, kind)
    Jbar = np.ones(N - 1) + 0.05 * np.arange(N - 1)
    epsbar = 0.1 * np.sin(np.arange(N))
    T = 2.5
    gJ, ge = G.ed_gradient(ens, Jbar, epsbar, w, T)
    fJ, fe = G.fd_gradient(lambda a, b: G.loss_exact(ens, a, b, w, T), Jbar, epsbar, h=1e-5)
    g_all = np.concatenate([gJ, ge])
    f_all = np.concatenate([fJ, fe])
    assert np.linalg.norm(g_all - f_all) <= 1e-7 * np.linalg.norm(f_all)
    assert np.linalg.norm(f_all) > 1e-3


def test_taylor_map_gradient_matches_exact_gradient_for_small_steps():
    """With order 14 and dt = 0.05 the truncated map differs from the exact
    one by far less than the FD error, so the FD of ``loss_taylor`` must agree
    with the exact-evolution gradient (pins ``loss_taylor``)."""
    ens = make_ensemble(B.BOSON, N=5, R=2)
    site_w = np.array([0, 0, 1, 1, 1.0])
    w = G.diagonal_weights(ens.states, site_w, G.PRODUCT)
    Jbar, epsbar = np.ones(4), np.zeros(5)
    dt, steps = 0.05, 40
    gJ, ge = G.ed_gradient(ens, Jbar, epsbar, w, dt * steps)
    rs = np.random.default_rng(3)
    vJ, ve = rs.normal(size=4), rs.normal(size=5)
    d = G.fd_directional(lambda a, b: G.loss_taylor(ens, a, b, w, dt, steps, order=14),
                         Jbar, epsbar, vJ, ve, h=1e-5)
    exact = float(gJ @ vJ + ge @ ve)
    assert abs(d - exact) <= 1e-7 * max(1.0, abs(exact))
    assert abs(exact) > 1e-3


def test_diagonal_weights_forms():
    states = B.basis_states(3, 2, B.BOSON)
    w1 = G.diagonal_weights(states, [1, 2, 4], G.ONE_BODY)
    w2 = G.diagonal_weights(states, [1, 2, 4], G.PRODUCT)
    for k, (a, b) in enumerate(states):
        assert w1[k] == [1, 2, 4][a] + [1, 2, 4][b]
        assert w2[k] == [1, 2, 4][a] * [1, 2, 4][b]


def test_periodic_bond_operator_includes_wrap_bond():
    op = Hm.bond_operator(4, 1, 3, boundary=Hm.PERIODIC).toarray()
    assert op[3, 0] == 1 and op[0, 3] == 1 and op.sum() == 2
