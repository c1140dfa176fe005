"""GPU adjoint: gradients of the ensemble-averaged diagonal observable with
respect to the baseline hoppings and on-site energies, through the C ABI,
against the FP64 oracle (central differences of the oracle's truncated-
Taylor map with the same number of terms, and the Daleckii-Krein gradient
of the exact evolution), plus invariants that hold at any size."""

import numpy as np
import pytest

from oracle import basis as B
from oracle import gradients as G
from oracle import hamiltonian as Hm

from _helpers import gpu_plan, say

pytestmark = pytest.mark.gpu


def noise(N, R, seed, boundary="open", Jsig=0.1, eps=0.5):
    g = np.random.default_rng(seed)
    nb = N if boundary == "periodic" else N - 1
    return g.normal(0, Jsig, (R, nb)), g.uniform(-eps, eps, (R, N)), g.uniform(0.5, 1.5, R)


def gpu_grad(stat, boundary, N, R, dJ, deps, U, Jbar, epsbar, sites, dt, steps, order, ckpt, sw, kind,
             dtype="c128"):
    reals = [(N, Jbar + dJ[r], epsbar + deps[r], float(U[r])) for r in range(R)]
    plan = gpu_plan(m=2, statistics=stat, boundary=boundary, interaction="onsite", dtype=dtype, reals=reals,
                    dt=dt, order=order, tol=0.0, sites=sites)
    return plan, plan.gradient(steps, ckpt, sw, kind)


@pytest.mark.parametrize("stat,kind,boundary", [("boson", "product", "open"),
                                                ("distinguishable", "one_body", "open"),
                                                ("distinguishable", "product", "periodic")])
def test_gradient_matches_finite_differences_c128(stat, kind, boundary):
    say(f"case: adjoint c128 {stat} {kind} {boundary} N=9 R=3, 30 steps, ckpt 7")
    N, R, dt, steps, order, ckpt = 9, 3, 0.05, 30, 10, 7
    dJ, deps, U = noise(N, R, 1, boundary)
    nb = dJ.shape[1]
    Jbar = 1.0 + 0.05 * np.arange(nb)
    epsbar = 0.1 * np.cos(np.arange(N))
    sw = np.linspace(-1, 1, N) if kind == "one_body" else (np.arange(N) >= 5).astype(float)
    sites = [3, 4]
    plan, (loss, gJ, gE) = gpu_grad(stat, boundary, N, R, dJ, deps, U, Jbar, epsbar, sites, dt, steps, order,
                                    ckpt, sw, kind)
    ens = G.Ensemble(N, 2, stat, dJ, deps, U, sites, boundary=boundary)
    w = G.diagonal_weights(ens.states, sw, G.PRODUCT if kind == "product" else G.ONE_BODY)
    fn = lambda a, b: G.loss_taylor(ens, a, b, w, dt, steps, order)  # noqa: E731
    l0 = fn(Jbar, epsbar)
    fJ, fE = G.fd_gradient(fn, Jbar, epsbar, h=1e-5)
    g_all, f_all = np.concatenate([gJ, gE]), np.concatenate([fJ, fE])
    rel = np.linalg.norm(g_all - f_all) / np.linalg.norm(f_all)
    say(f"  loss {loss:.12f} (oracle {l0:.12f}); |g - g_fd| / |g_fd| = {rel:.2e}")
    assert abs(loss - l0) < 1e-12
    assert rel <= 1e-6
    # the state after the call is psi(T)
    assert plan.stats().steps_done == steps


@pytest.mark.parametrize("m,stat,boundary,N", [(1, "distinguishable", "open", 150),
                                                (1, "distinguishable", "periodic", 150),
                                                (2, "distinguishable", "periodic", 70),
                                                (2, "boson", "open", 130)])
def test_gradient_several_bands_c128(m, stat, boundary, N):
    """Lattices wider than one backward band (62 output columns): the
    derivative of the loss along two random directions of (Jbar, epsbar)
    equals the central difference of the oracle's truncated-Taylor loss
    (relative to |grad| |direction|: 1e-8), and the loss the oracle's."""
    say(f"case: adjoint c128 m={m} {stat} {boundary} N={N} R=2, 30 steps, ckpt 7")
    R, dt, steps, order, ckpt = 2, 0.05, 30, 10, 7
    dJ, deps, U = noise(N, R, 4, boundary)
    nb = dJ.shape[1]
    Jbar = 1.0 + 0.05 * np.sin(np.arange(nb))
    epsbar = 0.1 * np.cos(np.arange(N))
    sw = np.linspace(-1, 1, N)
    sites = [N // 3] if m == 1 else [N // 3, N // 3 + 1]
    reals = [(N, Jbar + dJ[r], epsbar + deps[r], float(U[r])) for r in range(R)]
    plan = gpu_plan(m=m, statistics=stat, boundary=boundary, interaction="onsite", dtype="c128", reals=reals,
                    dt=dt, order=order, tol=0.0, sites=sites)
    loss, gJ, gE = plan.gradient(steps, ckpt, sw, "one_body")
    ens = G.Ensemble(N, m, stat, dJ, deps, U, sites, boundary=boundary)
    w = G.diagonal_weights(ens.states, sw, G.ONE_BODY)
    fn = lambda a, b: G.loss_taylor(ens, a, b, w, dt, steps, order)  # noqa: E731
    l0 = fn(Jbar, epsbar)
    g_all = np.concatenate([gJ, gE])
    rs = np.random.default_rng(5)
    worst = 0.0
    for _ in range(2):
        vJ, vE = rs.normal(size=nb), rs.normal(size=N)
        fd = G.fd_directional(fn, Jbar, epsbar, vJ, vE, h=1e-5)
        ad = float(gJ @ vJ + gE @ vE)
        worst = max(worst, abs(ad - fd) / (np.linalg.norm(g_all) * np.linalg.norm(np.concatenate([vJ, vE]))))
    say(f"  loss {loss:.12f} (oracle {l0:.12f}); directional error / (|g| |v|) = {worst:.2e}")
    assert abs(loss - l0) < 1e-12
    assert worst <= 1e-8


def test_gradient_matches_exact_evolution_gradient_reduced_c4():
    """Reduced gradient workload: two bosons on N=32, U=1, J noise 0.1,
    eps noise U[-0.5,0.5], 8 realisations, loss = probability that both are
    in nodes 24..31 at t = 20 (400 steps of dt = 0.05, checkpoints every 32).
    With 12 terms per step the truncated map is exact to ~1e-14 per step, so
    the Daleckii-Krein gradient of the exact evolution must agree to 1e-8."""
    say("case: reduced adjoint workload N=32 bosons R=8, 400 steps, ckpt 32, c128")
    N, R, dt, steps = 32, 8, 0.05, 400
    dJ, deps, _ = noise(N, R, 2)
    U = np.ones(R)
    Jbar, epsbar = np.ones(N - 1), np.zeros(N)
    sw = (np.arange(N) >= 24).astype(float)
    sites = [19, 20]
    _, (loss, gJ, gE) = gpu_grad("boson", "open", N, R, dJ, deps, U, Jbar, epsbar, sites, dt, steps, 12, 32, sw,
                                 "product")
    ens = G.Ensemble(N, 2, "boson", dJ, deps, U, sites)
    w = G.diagonal_weights(ens.states, sw, G.PRODUCT)
    eJ, eE = G.ed_gradient(ens, Jbar, epsbar, w, dt * steps)
    le = G.loss_exact(ens, Jbar, epsbar, w, dt * steps)
    e_all, g_all = np.concatenate([eJ, eE]), np.concatenate([gJ, gE])
    rel = np.linalg.norm(g_all - e_all) / np.linalg.norm(e_all)
    say(f"  loss {loss:.6e} (exact {le:.6e}); |g - g_ED| / |g_ED| = {rel:.2e}; |grad| = {np.linalg.norm(e_all):.3e}")
    assert abs(loss - le) <= 1e-10 * max(1.0, abs(le))
    assert rel <= 1e-8


def test_gradient_c64_against_oracle():
    """complex64 state and adjoint vectors, FP64 contractions: relative
    error of the gradient against the FP64 finite differences <= 1e-4."""
    say("case: adjoint c64 bosons N=12 R=4, 60 steps")
    N, R, dt, steps, order = 12, 4, 0.05, 60, 7
    dJ, deps, U = noise(N, R, 3)
    Jbar, epsbar = np.ones(N - 1), np.zeros(N)
    sw = (np.arange(N) >= 7).astype(float)
    sites = [5, 6]
    _, (loss, gJ, gE) = gpu_grad("boson", "open", N, R, dJ, deps, U, Jbar, epsbar, sites, dt, steps, order, 16,
                                 sw, "product", dtype="c64")
    ens = G.Ensemble(N, 2, "boson", dJ, deps, U, sites)
    w = G.diagonal_weights(ens.states, sw, G.PRODUCT)
    fn = lambda a, b: G.loss_taylor(ens, a, b, w, dt, steps, order)  # noqa: E731
    fJ, fE = G.fd_gradient(fn, Jbar, epsbar, h=1e-5)
    g_all, f_all = np.concatenate([gJ, gE]), np.concatenate([fJ, fE])
    rel = np.linalg.norm(g_all - f_all) / np.linalg.norm(f_all)
    say(f"  c64: |g - g_fd| / |g_fd| = {rel:.2e}, loss err {abs(loss - fn(Jbar, epsbar)):.2e}")
    assert rel <= 1e-4


def test_autograd_function_and_checkpoint_invariance():
    import torch
    from paper_1612_00746_amd.autograd import EnsembleLoss, NoisyWalk
    say("case: torch.autograd.Function + checkpoint spacing invariance")
    N, R, dt, steps = 10, 3, 0.05, 24
    dJ, deps, U = noise(N, R, 4)
    sw = (np.arange(N) >= 6).astype(float)
    reals = [(N, 1 + dJ[r], deps[r], float(U[r])) for r in range(R)]
    plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype="c128", reals=reals,
                    dt=dt, order=10, tol=0.0)
    model = NoisyWalk(plan, dJ, deps, U, [4, 5], steps, 5, sw, "product")
    Jbar = torch.ones(N - 1, dtype=torch.float64, requires_grad=True)
    epsbar = torch.zeros(N, dtype=torch.float64, requires_grad=True)
    L = EnsembleLoss.apply(Jbar, epsbar, model)
    (3.0 * L).backward()
    grads = []
    for ckpt in (1, 5, 24, 100):
        plan.init_product_state([4, 5])
        loss, gJ, gE = plan.gradient(steps, ckpt, sw, "product")
        grads.append(np.concatenate([gJ, gE]))
        assert abs(loss - float(L)) < 1e-14
    for gr in grads[1:]:
        assert np.array_equal(gr, grads[0])   # identical arithmetic for any spacing
    assert np.max(np.abs(Jbar.grad.numpy() - 3.0 * grads[0][:N - 1])) < 1e-15
    assert np.max(np.abs(epsbar.grad.numpy() - 3.0 * grads[0][N - 1:])) < 1e-15


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_size_gradient_workload(dtype):
    """Gradient workload at full size: two bosons on N=256, U=1, 512
    realisations, loss = probability both in nodes 192..255 at t=20, 400
    steps, checkpoints every 32.  Checks at this size: a uniform shift of all
    on-site energies only adds a global phase, so sum_i dL/deps_i = 0; the
    directional derivative along a random direction matches a central
    difference of the GPU's own forward map (FP64)."""
    import time
    from workloads import C4
    w = C4(dtype)
    say(f"case: {w.name} {dtype} R={w.R} N={w.N} steps={w.n_steps}")
    reals = w.all_realizations()
    plan = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype=dtype, reals=reals,
                    dt=w.dt, tol=w.tol, sites=list(w.start))
    sw = (np.arange(w.N) >= 192).astype(float)
    t0 = time.perf_counter()
    loss, gJ, gE = plan.gradient(w.n_steps, 32, sw, "product")
    el = time.perf_counter() - t0
    say(f"  loss {loss:.6e}, |dL/dJ| {np.linalg.norm(gJ):.3e}, |dL/deps| {np.linalg.norm(gE):.3e}, "
        f"sum dL/deps {gE.sum():.2e}, {el:.2f} s per gradient, order {plan.orders().max()}")
    assert np.all(np.isfinite(gJ)) and np.all(np.isfinite(gE))
    scale = np.linalg.norm(gE) + 1e-300
    assert abs(gE.sum()) <= (1e-9 if dtype == "c128" else 1e-4) * scale * np.sqrt(w.N)
    if dtype == "c128":
        rs = np.random.default_rng(7)
        vJ, vE = rs.normal(size=w.N - 1), rs.normal(size=w.N)
        h = 1e-4

        def fwd(sgn):
            shifted = [(N, J + sgn * h * vJ, e + sgn * h * vE, U) for (N, J, e, U) in reals]
            p = gpu_plan(m=2, statistics="boson", boundary="open", interaction="onsite", dtype=dtype,
                         reals=shifted, dt=w.dt, tol=w.tol, sites=list(w.start))
            p.propagate(w.n_steps)
            return p.loss(sw, "product")
        fd = (fwd(+1) - fwd(-1)) / (2 * h)
        ad = float(gJ @ vJ + gE @ vE)
        say(f"  directional: adjoint {ad:.10e} vs central difference {fd:.10e}")
        assert abs(ad - fd) <= 1e-6 * max(abs(fd), 1e-12)
