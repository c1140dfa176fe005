"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/ctqw.h, validates problems, selects
Taylor orders and reports layouts and sizes without touching a device."""

import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from _helpers import reference_order

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctqw.h")

lib_path = os.path.join(ROOT, "paper_1612_00746_amd", "libctqw.so")
pytestmark = pytest.mark.skipif(not os.path.exists(lib_path), reason="libctqw.so not built")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctqw_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_1612_00746_amd import _lib as L
    lib = L.load()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), "binding and header disagree"


def make(**kw):
    from paper_1612_00746_amd import Plan, make_problem
    args = dict(m=2, R=3, n_sites=8, dt=0.05, taylor_tol=1e-12)
    args.update(kw)
    pr, keep = make_problem(**args)
    plan = Plan(pr)
    plan._keep.append(keep)
    return plan


def status_of(fn):
    from paper_1612_00746_amd import CtqwError
    try:
        fn()
    except CtqwError as e:
        return e.status
    return 0


@pytest.mark.parametrize("kw,status", [
    (dict(m=0), 1), (dict(m=4), 1), (dict(m=3, statistics="boson"), 2), (dict(m=3, n_sites=[8, 8, 9]), 2),
    (dict(m=3, n_sites=2000), 2),
    (dict(n_sites=1), 1), (dict(R=0), 1),
    (dict(dt=0.0), 1), (dict(dt=float("nan")), 1), (dict(dt=-1.0), 1),
    (dict(taylor_tol=0.0), 1),
    (dict(boundary="periodic", n_sites=2), 1),
    (dict(statistics="boson", boundary="periodic"), 2),
])
def test_plan_create_validation(kw, status):
    assert status_of(lambda: make(**kw)) == status


def test_invalid_enum_and_null():
    from paper_1612_00746_amd import _lib as L
    lib = L.load()
    from paper_1612_00746_amd import make_problem
    pr, _ = make_problem(2, 2, 8, 0.1, taylor_tol=1e-10)
    pr.dtype = 7
    h = L.PlanP()
    assert lib.ctqw_plan_create(C.byref(pr), C.byref(h)) == L.ERR_INVALID_ARG
    assert b"dtype" in lib.ctqw_last_error(None)
    assert lib.ctqw_plan_create(None, C.byref(h)) == L.ERR_INVALID_ARG


def draw(plan_N, R, nb, seed=0):
    g = np.random.default_rng(seed)
    J = 1 + 0.1 * g.standard_normal(R * nb)
    eps = g.uniform(-0.5, 0.5, R * plan_N)
    U = g.uniform(0, 2, R)
    return J, eps, U


def test_set_params_rejects_nonfinite_and_keeps_state():
    plan = make()
    J, eps, U = draw(8, 3, 7)
    bad = J.copy()
    bad[4] = np.inf
    assert status_of(lambda: plan.set_params(bad, eps, U)) == 1
    plan.set_params(J, eps, U)
    o = plan.orders()
    assert status_of(lambda: plan.set_params(J, eps, np.array([0, np.nan, 0.0]))) == 1
    assert np.array_equal(plan.orders(), o)


@pytest.mark.parametrize("m,periodic,tol,dt", [(2, False, 1e-14, 0.05), (2, True, 1e-7, 0.05),
                                               (1, False, 1e-12, 0.2), (2, False, 1e-10, 0.01)])
def test_apriori_taylor_orders(m, periodic, tol, dt):
    N, R = 12, 5
    plan = make(m=m, R=R, n_sites=N, dt=dt, taylor_tol=tol, boundary="periodic" if periodic else "open",
                dtype="c128")
    nb = N if periodic else N - 1
    J, eps, U = draw(N, R, nb, seed=3)
    plan.set_params(J, eps, U)
    got = plan.orders()
    for r in range(R):
        assert got[r] == reference_order(J[r * nb:(r + 1) * nb], eps[r * N:(r + 1) * N], U[r], m, dt, tol)


def test_fixed_order_and_cap():
    plan = make(taylor_order=5, taylor_tol=0.0)
    J, eps, U = draw(8, 3, 7)
    plan.set_params(J, eps, U)
    assert list(plan.orders()) == [5, 5, 5]
    plan2 = make(dt=2.0, taylor_tol=1e-14)
    assert status_of(lambda: plan2.set_params(J, eps, U)) == 5   # NOT_CONVERGED
    plan3 = make(taylor_order=45, taylor_tol=0.0)      # above the default cap of 40
    assert status_of(lambda: plan3.set_params(J, eps, U)) == 5
    plan4 = make(taylor_order=30, taylor_tol=0.0, taylor_max_order=25)
    assert status_of(lambda: plan4.set_params(J, eps, U)) == 5


def test_orders_above_the_fused_depth_run_in_passes():
    """Order 20 (above the fused pipeline's 12 / 16 terms) is accepted and
    laid out for chunked passes: 64-column bands with a halo of the pass
    depth (8 terms complex64, 4 complex128) and three extra state buffers;
    the chunked launch flag forces the same layout for low orders."""
    for dtype, K, esz in (("c64", 8, 8), ("c128", 4, 16)):
        N = 200
        plan = make(R=1, n_sites=N, taylor_order=20, taylor_tol=0.0, dtype=dtype)
        plan.set_params(np.ones(N - 1), np.zeros(N), np.zeros(1))
        bands = -(-(N - (64 - K)) // (64 - 2 * K)) + 1
        assert plan.work_items()[0] == bands, dtype
        fused = make(R=1, n_sites=N, taylor_order=6, taylor_tol=0.0, dtype=dtype)
        fused.set_params(np.ones(N - 1), np.zeros(N), np.zeros(1))
        fused.set_launch(row_segments=1)   # the chunked layout has no row segments
        sb_f, ws_f = fused.sizes()
        fused.set_launch(chunked=1)
        sb_c, ws_c = fused.sizes()
        assert ws_c - ws_f >= 3 * N * N * esz


def test_layout_sizes_groups_uneven():
    Ns = [16, 40, 16, 70, 40]
    plan = make(R=5, n_sites=Ns, statistics="boson", dtype="c64")
    nbs = [n - 1 for n in Ns]
    g = np.random.default_rng(1)
    plan.set_params(1 + 0.1 * g.standard_normal(sum(nbs)), g.uniform(-1, 1, sum(Ns)), np.ones(5))
    off = plan.layout()
    assert list(np.diff(off)) == [n * (n + 1) // 2 for n in Ns]
    sb, wb = plan.sizes()
    assert sb == off[-1] * 8 and wb > 0
    assert list(plan.groups()) == [16, 40, 70]
    items, _ = plan.work_items()
    assert items >= 5


def test_band_partition_covers_columns_once():
    """Each realisation's bands must cover every column exactly once; the
    number of bands follows from the window (64 per lane column) and halo."""
    for P, N, expect in [(1, 64, 1), (1, 65, 2), (1, 200, 4), (2, 128, 1), (2, 300, 3)]:
        plan = make(R=1, n_sites=N, taylor_order=7, taylor_tol=0.0)
        plan.set_launch(cols_per_lane=P, row_segments=1)
        plan.set_params(np.ones(N - 1), np.zeros(N), np.zeros(1))
        assert plan.work_items()[0] == expect, (P, N)


def test_few_bands_split_their_rows():
    """A batch with few bands has each band's rows split into segments of
    at least twice the halo (the Taylor order) output rows; row_segments
    caps the count, 1 switches the split off, and the default splits only
    small batches."""
    N, n = 200, 7
    plan = make(R=1, n_sites=N, taylor_order=n, taylor_tol=0.0)
    plan.set_launch(cols_per_lane=1, row_segments=1)
    plan.set_params(np.ones(N - 1), np.zeros(N), np.zeros(1))
    bands = plan.work_items()[0]
    assert bands == 4
    for cap in (2, 5, 16):
        plan.set_launch(row_segments=cap)
        assert plan.work_items()[0] == bands * min(cap, N // (2 * n)), cap
    plan.set_launch(row_segments=0)
    assert plan.work_items()[0] == bands * min(16, N // (2 * n))
    # three-particle and one-particle plans are never split
    one = make(R=1, m=1, n_sites=N, taylor_order=n, taylor_tol=0.0)
    one.set_launch(cols_per_lane=1)
    one.set_params(np.ones(N - 1), np.zeros(N), np.zeros(1))
    assert one.work_items()[0] == 4
    from paper_1612_00746_amd import CtqwError
    with pytest.raises(CtqwError):
        plan.set_launch(row_segments=17)
    with pytest.raises(CtqwError):
        plan.set_launch(row_segments=-1)


def test_bind_requires_valid_buffers_without_touching_device():
    from paper_1612_00746_amd import _lib as L
    plan = make()
    lib = plan.lib
    assert lib.ctqw_bind(plan.h, None, None, 0, None, 0, None) == L.ERR_STATE   # params not set
    J, eps, U = draw(8, 3, 7)
    plan.set_params(J, eps, U)
    assert lib.ctqw_bind(plan.h, None, None, 0, None, 0, None) == L.ERR_INVALID_ARG
    out = np.zeros(4)
    assert lib.ctqw_propagate(plan.h, 1, 0, 0, None) == L.ERR_STATE
    assert lib.ctqw_init_product_state(plan.h, np.zeros(2, np.int32).ctypes.data_as(L.i32p), 0) == L.ERR_STATE
    assert lib.ctqw_observe(plan.h, 1, out.ctypes.data_as(L.dp)) == L.ERR_STATE


def test_launch_validation():
    from paper_1612_00746_amd import CtqwError
    plan = make()
    with pytest.raises(CtqwError):
        plan.set_launch(cols_per_lane=3)
    with pytest.raises(CtqwError):
        plan.set_launch(waves_per_block=8)
    plan.set_launch(cols_per_lane=2, persistent=1)
    assert plan.get_launch().cols_per_lane == 2


def test_status_strings():
    from paper_1612_00746_amd import _lib as L
    lib = L.load()
    for s in range(8):
        assert lib.ctqw_status_string(s)
    assert lib.ctqw_version().startswith(b"ctqw")


def test_gradient_entry_points_validate_on_host():
    from paper_1612_00746_amd import _lib as L
    plan = make(R=2, n_sites=8, statistics="boson", taylor_order=6, taylor_tol=0.0)
    J, eps, U = draw(8, 2, 7)
    plan.set_params(J, eps, U)
    lib = plan.lib
    b = np.zeros(1, dtype=np.int64)
    assert lib.ctqw_gradient_workspace(plan.h, 40, 8, b.ctypes.data_as(L.i64p)) == 0
    esz = 16
    S = ((8 * 9 // 2) * 2 * esz + 255) // 256 * 256
    # 5 checkpoints + 7 segment states + 5 Taylor vectors + 2 Horner + 2 adjoint states
    assert b[0] >= (5 + 7 + 5 + 4) * S
    assert lib.ctqw_gradient_workspace(plan.h, 40, 0, b.ctypes.data_as(L.i64p)) == L.ERR_INVALID_ARG
    w = np.ones(8)
    out = np.zeros(16)
    loss = np.zeros(1)
    dp = L.dp
    assert lib.ctqw_gradient(plan.h, 10, 2, 5, w.ctypes.data_as(dp), None, 0, loss.ctypes.data_as(dp),
                             out.ctypes.data_as(dp), out.ctypes.data_as(dp)) == L.ERR_INVALID_ARG
    assert lib.ctqw_backward(plan.h, 1, w.ctypes.data_as(dp), C.c_void_p(256), 1 << 30, loss.ctypes.data_as(dp),
                             out.ctypes.data_as(dp), out.ctypes.data_as(dp)) == L.ERR_STATE
    uneven = make(R=2, n_sites=[8, 10], taylor_order=6, taylor_tol=0.0)
    uneven.set_params(np.ones(7 + 9), np.zeros(18), np.zeros(2))
    assert lib.ctqw_forward_ckpt(uneven.h, 4, 2, C.c_void_p(256), 1 << 30) == L.ERR_UNSUPPORTED
    renorm = make(R=2, n_sites=8, taylor_order=6, taylor_tol=0.0, renormalize=True)
    renorm.set_params(J, eps, U)
    assert lib.ctqw_forward_ckpt(renorm.h, 4, 2, C.c_void_p(256), 1 << 30) == L.ERR_UNSUPPORTED
    # the adjoint passes address a realisation's state through one buffer
    # resource: states of 2^31 bytes and more are refused before device work
    for dtype, n in (("c64", 16384), ("c128", 11586)):
        big = make(R=1, n_sites=n, taylor_order=6, taylor_tol=0.0, dtype=dtype)
        big.set_params(np.ones(n - 1), np.zeros(n), np.zeros(1))
        assert lib.ctqw_forward_ckpt(big.h, 4, 2, C.c_void_p(256), 1 << 40) == L.ERR_UNSUPPORTED, dtype
        assert b"2 GiB" in lib.ctqw_last_error(big.h), dtype


@pytest.mark.parametrize("boundary", ["open", "periodic"])
def test_draw_params_match_the_oracle_generator(boundary):
    """Library draws (Philox4x32-10, host side) against the oracle's own
    generator: uniform draws bit for bit, Box-Muller normals within 2 ulp
    (libm's log/cos), for an uneven batch with baselines; the orders follow
    from the drawn values."""
    from oracle import noise
    Ns = [8, 13, 8, 21]
    plan = make(R=4, n_sites=Ns, boundary=boundary, dtype="c64", taylor_tol=1e-7)
    nbmax = max(Ns) if boundary == "periodic" else max(Ns) - 1
    g = np.random.default_rng(5)
    Jb, Eb = 1 + 0.05 * g.standard_normal(nbmax), g.uniform(-0.2, 0.2, max(Ns))
    kw = dict(J_base=Jb, eps_base=Eb, U_base=1.5, J_noise=("normal", 0.0, 0.1),
              eps_noise=("uniform", -0.5, 0.5), U_noise=("uniform", 0.0, 4.0), seed=12345678901)
    plan.draw_params(**kw)
    J, eps, U = plan.get_params()
    J0, eps0, U0 = noise.draw_params(Ns, boundary == "periodic", **kw)
    assert np.array_equal(eps, eps0) and np.array_equal(U, U0)
    np.testing.assert_array_max_ulp(J, np.array(J0), maxulp=2)
    nb = [n if boundary == "periodic" else n - 1 for n in Ns]
    jo = np.cumsum([0] + nb)
    eo = np.cumsum([0] + Ns)
    o = plan.orders()
    for r in range(4):
        assert o[r] == reference_order(J[jo[r]:jo[r + 1]], eps[eo[r]:eo[r + 1]], U[r], 2, 0.05, 1e-7)
    # defaults: no noise -> J = 1, eps = 0, U = U_base
    plan.draw_params(U_base=0.5)
    J, eps, U = plan.get_params()
    assert np.all(J == 1.0) and np.all(eps == 0.0) and np.all(U == 0.5)


def test_draw_params_validation():
    from paper_1612_00746_amd import _lib as L
    plan = make(R=2, n_sites=8)
    assert status_of(lambda: plan.draw_params(J_noise=("uniform", 0.0, float("nan")))) == 1
    bad = L.Noise(7, 0.0, 1.0)
    assert plan.lib.ctqw_draw_params(plan.h, None, None, 0.0, C.byref(bad), None, None, 0) == L.ERR_INVALID_ARG
    assert status_of(lambda: plan.draw_params(U_base=float("inf"))) == 1


def reference_band_count(N, h, W, align_cols, pairs):
    """Bands of one open chain by the documented rule: windows of W columns
    with a halo of h, boundaries moved down to multiples of align_cols
    columns where a band keeps an output column, window starts made even
    for paired (two-column) lanes."""
    lo, n = 0, 0
    while lo < N:
        w0 = max(0, lo - h)
        if pairs and w0 % 2:
            w0 -= 1
        if w0 + W > N:
            w0 = max(0, N - W)
        w1 = min(N, w0 + W)
        if w1 == N:
            hi = N
        else:
            hi = w1 - h
            a = (hi // align_cols) * align_cols
            hi = a if a > lo else hi
        assert hi > lo
        n += 1
        lo = hi
    return n


@pytest.mark.parametrize("P", [1, 2])
@pytest.mark.parametrize("align", [0, 64, 128])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_band_boundaries_follow_the_alignment(P, align, dtype):
    """Work items per step for open chains of several lengths at order 7
    match the band rule; alignment never changes the number of items."""
    Ns = [64, 96, 300, 999, 1024]
    plan = make(R=len(Ns), n_sites=Ns, taylor_order=7, taylor_tol=0.0, dtype=dtype)
    plan.set_launch(cols_per_lane=P, band_align=align, row_segments=1)
    nb = sum(N - 1 for N in Ns)
    J, _, U = draw(1, len(Ns), nb)
    eps = np.zeros(sum(Ns))
    plan.set_params(J, eps, U)
    amp = 8 if dtype == "c64" else 16
    cols = max(1, align // amp)
    pairs = P == 2 and dtype == "c64"
    want = 0
    for N in Ns:
        # the largest power-of-two fraction of the alignment adding no band
        base = reference_band_count(N, 7, 64 * P, 1, pairs)
        a = cols
        while a > 1 and reference_band_count(N, 7, 64 * P, a, pairs) > base:
            a //= 2
        want += reference_band_count(N, 7, 64 * P, a, pairs)
    items, _ = plan.work_items()
    assert items == want
    plan.set_launch(cols_per_lane=P, band_align=0)
    assert plan.work_items()[0] == items


def test_band_align_values_are_checked():
    plan = make()
    assert status_of(lambda: plan.set_launch(band_align=96)) == 1
    assert status_of(lambda: plan.set_launch(band_align=-1)) == 1


def test_rk4_method_is_the_degree_four_step():
    """method="rk4" runs Alg. 2 as the degree-4 Taylor step: every
    realisation takes CTQW_RK4_ORDER terms, and the constant matches the
    header."""
    from paper_1612_00746_amd import _lib as L, make_problem
    text = open(HEADER).read()
    m = re.search(r"#define CTQW_RK4_ORDER (\d+)", text)
    assert m and int(m.group(1)) == L.RK4_ORDER == 4
    plan = make(method="rk4", taylor_tol=0.0)
    J, eps, U = draw(8, 3, 7)
    plan.set_params(J, eps, U)
    assert list(plan.orders()) == [4, 4, 4]
    with pytest.raises(ValueError):
        make_problem(2, 3, 8, 0.05, method="rk4", taylor_tol=1e-7)
    with pytest.raises(ValueError):
        make_problem(2, 3, 8, 0.05, method="euler")


def test_switching_noise_orders_and_validation():
    """With switching noise of amplitude a the a-priori orders take
    |Jbar| + a on every bond; bad amplitudes and rates are rejected."""
    N, R = 12, 4
    plan = make(R=R, n_sites=N, dt=0.05, taylor_tol=1e-10, dtype="c128")
    J, eps, U = draw(N, R, N - 1, seed=8)
    plan.set_params(J, eps, U)
    static = plan.orders().copy()
    plan.set_telegraph(0.8, 3.0, 5)
    got = plan.orders()
    for r in range(R):
        Jr = np.abs(J[r * (N - 1):(r + 1) * (N - 1)]) + 0.8
        assert got[r] == reference_order(Jr, eps[r * N:(r + 1) * N], U[r], 2, 0.05, 1e-10)
    assert np.all(got >= static) and np.any(got > static)
    assert status_of(lambda: plan.set_telegraph(-0.1, 1.0, 0)) == 1
    assert status_of(lambda: plan.set_telegraph(0.1, float("nan"), 0)) == 1
    plan.set_telegraph(0.0, 0.0, 0)
    assert np.array_equal(plan.orders(), static)


def test_density_matrix_arguments_are_checked():
    """Workspace size of a group's density matrix (real and imaginary
    planes of D x R_g padded to whole 128-row tiles and 16-realisation
    stages for complex64), group range and the state of the plan (not
    bound) are checked on the host."""
    import ctypes as C2
    plan = make(R=3, n_sites=[6, 8, 6], dtype="c64", taylor_tol=1e-7)
    J, eps, U = draw(8, 3, 7)
    plan.set_params(np.concatenate([J[0:5], J[7:14], J[14:19]]), np.concatenate([eps[0:6], eps[8:16], eps[16:22]]), U)
    ws = C2.c_int64()
    assert plan.lib.ctqw_density_workspace(plan.h, 0, C2.byref(ws)) == 0
    assert ws.value == 2 * 128 * 16 * 4      # N = 6: D = 36 -> 128 rows, two realisations -> 16, two FP32 planes
    assert plan.lib.ctqw_density_workspace(plan.h, 1, C2.byref(ws)) == 0
    assert ws.value == 2 * 128 * 16 * 4
    assert plan.lib.ctqw_density_workspace(plan.h, 2, C2.byref(ws)) == 1
    buf = C2.create_string_buffer(16384)
    assert plan.lib.ctqw_density_matrix(plan.h, 0, buf, 36, 0, buf, 16384) == 7   # STATE: not bound
    assert plan.lib.ctqw_density_matrix(plan.h, 0, buf, 20, 0, buf, 16384) == 1   # ld below D
    assert plan.lib.ctqw_density_matrix(plan.h, 0, buf, 36, 0, buf, 16383) == 1   # workspace too small


# ---------------------------------------------------------------- general graphs
@pytest.mark.parametrize("shape,periodic", [((5, 7), False), ((3, 4, 5), True), ((2, 6), True), ((1, 4), False)])
def test_lattice_edges_match_the_oracle_bonds(shape, periodic):
    from paper_1612_00746_amd import lattice_edges
    from oracle import graph as G
    got = sorted(map(tuple, lattice_edges(shape, periodic).tolist()))
    assert got == G.lattice_bonds(shape, periodic)


def test_ell_tables_rebuild_the_oracle_hamiltonian():
    """A random graph with degrees 0 to several (an isolated node
    included): the ELL tables, read back as a matrix, equal the oracle's
    off-diagonal H for every realisation."""
    from paper_1612_00746_amd import ell_tables
    from oracle import graph as G
    g = np.random.default_rng(7)
    n = 30
    pairs = {(int(a), int(b)) for a, b in g.integers(0, n - 1, (80, 2)) if a != b}
    edges = sorted((min(a, b), max(a, b)) for a, b in pairs)
    edges = sorted(set(edges))
    J = g.standard_normal((3, len(edges)))
    nbr, hop = ell_tables(n, np.array(edges), J)
    assert nbr.flags.c_contiguous and hop.flags.c_contiguous
    assert nbr.shape[0] == max(np.bincount(np.array(edges).ravel(), minlength=n))
    assert np.all(nbr[:, n - 1] == -1)
    for r in range(3):
        M = np.zeros((n, n))
        for k in range(nbr.shape[0]):
            for i in range(n):
                if nbr[k, i] >= 0:
                    M[i, nbr[k, i]] += hop[r, k, i]
        ref = G.hamiltonian(n, edges, J[r], np.zeros(n)).toarray()
        assert np.array_equal(M, ref)


def test_ell_tables_reject_bad_bonds():
    """ctqw_graph_tables refuses self-loops, repeated bonds (either
    orientation) and nodes out of range with INVALID_ARG."""
    from paper_1612_00746_amd import CtqwError, ell_tables
    for edges in ([(0, 0)], [(0, 1), (1, 0)], [(0, 5)], [(-1, 2)]):
        with pytest.raises(CtqwError) as e:
            ell_tables(4, np.array(edges), np.ones((1, len(edges))))
        assert e.value.status == 1


def test_graph_tables_sizes_and_one_particle_onsite():
    """The size query returns the state count and width of each case
    (n, n^2, n(n+1)/2, n(n-1)/2 states; width = largest degree, doubled for
    pairs), and one particle's on-site table is eps itself."""
    from paper_1612_00746_amd import _lib as L
    from paper_1612_00746_amd import graph_tables, lattice_edges
    lib = L.load()
    edges = np.ascontiguousarray(lattice_edges((3, 4)), dtype=np.int32)
    n = 12
    for m, stat, D in ((1, 0, n), (2, 0, n * n), (2, 1, n * (n + 1) // 2), (2, 2, n * (n - 1) // 2)):
        ns, w = C.c_int32(), C.c_int32()
        assert lib.ctqw_graph_tables(n, len(edges), C.c_void_p(edges.ctypes.data), m, stat, 0, None, None, None,
                                     C.byref(ns), C.byref(w), None, None, None) == 0
        assert ns.value == D and w.value == 4 * m
    eps = np.random.default_rng(3).uniform(-1, 1, (2, n))
    nbr, hop, onsite = graph_tables(n, edges, np.ones((2, len(edges))), eps)
    assert np.array_equal(onsite, eps)


@pytest.mark.parametrize("kw,status", [
    (dict(n_nodes=0), 1), (dict(R=0), 1), (dict(width=-1), 1), (dict(order=0), 1), (dict(order=65), 1),
    (dict(n_steps=-1), 1), (dict(dt=float("nan")), 1), (dict(ws=10), 1), (dict(psi=None), 1), (dict(dtype=2), 1),
])
def test_graph_evolve_validation(kw, status):
    """Invalid requests are refused on the host, before any device work."""
    from paper_1612_00746_amd import _lib as L
    lib = L.load()
    a = dict(n_nodes=8, width=2, nbr=C.c_void_p(16), hop=C.c_void_p(16), onsite=C.c_void_p(16), R=2, dt=0.1,
             order=4, n_steps=1, psi=C.c_void_p(16), ws=C.c_void_p(16), ws_bytes=3 * 8 * 2 * 16, dtype=1)
    if "ws" in kw:
        a["ws_bytes"] = kw.pop("ws")
    a.update(kw)
    st = lib.ctqw_graph_evolve(a["n_nodes"], a["width"], a["nbr"], a["hop"], a["onsite"], a["R"], a["dtype"],
                               a["dt"], a["order"], a["n_steps"], a["psi"], a["ws"], a["ws_bytes"], None, None)
    assert st == status
    b = C.c_int64()
    assert lib.ctqw_graph_workspace(8, 2, 1, C.byref(b)) == 0 and b.value == 3 * 8 * 2 * 16
    assert lib.ctqw_graph_workspace(8, 2, 0, C.byref(b)) == 0 and b.value == 3 * 8 * 2 * 8


@pytest.mark.parametrize("kw,status", [
    (dict(Lx=0), 1), (dict(Ly=0), 1), (dict(R=0), 1), (dict(order=0), 1), (dict(order=13), 2),
    (dict(order=11, dtype=1), 2), (dict(px=1, Lx=2), 1), (dict(py=1, Ly=2), 1), (dict(n_steps=-1), 1),
    (dict(dt=float("inf")), 1), (dict(ws=64), 1), (dict(psi=None), 1), (dict(dtype=3), 1),
])
def test_lattice_evolve_validation(kw, status):
    """Invalid requests to the two-dimensional lattice path are refused on
    the host before any device work (1: INVALID_ARG, 2: UNSUPPORTED)."""
    from paper_1612_00746_amd import _lib as L
    lib = L.load()
    a = dict(Lx=70, Ly=9, px=0, py=0, R=2, tab=C.c_void_p(256), dtype=0, dt=0.05, order=10, n_steps=1,
             psi=C.c_void_p(256), ws=None, ws_ptr=C.c_void_p(256))
    a.update(kw)
    b = C.c_int64()
    ok = lib.ctqw_lattice_workspace(a["Lx"], a["Ly"], a["R"], a["dtype"], a["order"], a["px"], C.byref(b))
    ws_bytes = a["ws"] if a["ws"] is not None else (b.value if ok == 0 else 1 << 20)
    st = lib.ctqw_lattice_evolve(a["Lx"], a["Ly"], a["px"], a["py"], a["R"], a["tab"], a["tab"], a["tab"], a["dtype"],
                                 a["dt"], a["order"], a["n_steps"], a["psi"], a["ws_ptr"], ws_bytes, None, None)
    assert st == status


def test_lattice_workspace_holds_a_state_the_tables_and_the_partials():
    """Workspace of the lattice path: a second state buffer, three dt-scaled
    tables and one FP64 norm partial per band and realisation, each region
    256-byte aligned (70 columns at order 10: two bands of 64 lanes)."""
    from paper_1612_00746_amd import _lib as L
    lib = L.load()
    b = C.c_int64()
    assert lib.ctqw_lattice_workspace(70, 9, 2, 0, 10, 0, C.byref(b)) == 0
    n = 70 * 9 * 2
    up = lambda x: (x + 255) // 256 * 256  # noqa: E731
    assert b.value == up(up(up(n * 8) + 3 * n * 4) + 2 * 2 * 8)
    assert lib.ctqw_lattice_workspace(70, 9, 2, 1, 8, 1, C.byref(b)) == 0
    assert b.value == up(up(up(n * 16) + 3 * n * 8) + 2 * 2 * 8)


@pytest.mark.parametrize("statistics", ["distinguishable", "boson", "fermion"])
def test_pair_tables_rebuild_the_oracle_pair_hamiltonian(statistics):
    """Two particles on a 3 x 4 lattice with noise and U: the pair-graph
    tables, read back as a matrix (ELL slots summed, on-site on the
    diagonal), equal the oracle's two-particle H for every realisation."""
    from paper_1612_00746_amd import lattice_edges, pair_tables
    from oracle import graph as G
    g = np.random.default_rng(10)
    edges = lattice_edges((3, 4))
    R = 2
    J, eps, U = 1 + 0.2 * g.standard_normal((R, len(edges))), g.uniform(-0.5, 0.5, (R, 12)), g.uniform(0.5, 2, R)
    nbr, hop, onsite = pair_tables(12, edges, J, eps, U, statistics)
    assert nbr.flags.c_contiguous and hop.flags.c_contiguous and onsite.flags.c_contiguous
    D = nbr.shape[1]
    bonds = [tuple(e) for e in edges.tolist()]
    for r in range(R):
        M = np.diag(onsite[r])
        for k in range(nbr.shape[0]):
            for i in range(D):
                if nbr[k, i] >= 0:
                    M[i, nbr[k, i]] += hop[r, k, i]
        ref = G.pair_hamiltonian(12, bonds, J[r], eps[r], U[r], statistics).toarray()
        assert np.allclose(M, ref, atol=1e-15)


def _rule_order(x, tol):
    n = 1
    while True:
        if x < n + 2 and x ** (n + 1) / math.factorial(n + 1) / (1 - x / (n + 2)) <= tol:
            return n
        n += 1


@pytest.mark.parametrize("statistics", [None, "distinguishable", "boson", "fermion"])
def test_graph_orders_follow_the_gershgorin_rule(statistics):
    """Orders of a noisy 5 x 4 lattice (one particle, or two with U)
    against the documented rule evaluated on the oracle's dense H
    (x = dt * largest absolute row sum)."""
    from paper_1612_00746_amd import ell_tables, graph_orders, lattice_edges, pair_tables
    from oracle import graph as G
    g = np.random.default_rng(11)
    edges = lattice_edges((5, 4))
    bonds = [tuple(e) for e in edges.tolist()]
    R, n, dt, tol = 4, 20, 0.07, 1e-9
    J = (1 + 0.3 * g.standard_normal((R, len(edges)))) * g.uniform(0.5, 2.0, (R, 1))
    eps, U = g.uniform(-1, 1, (R, n)), g.uniform(0, 3, R)
    if statistics is None:
        nbr, hop = ell_tables(n, edges, J)
        onsite = eps
        Hs = [G.hamiltonian(n, bonds, J[r], eps[r]) for r in range(R)]
    else:
        nbr, hop, onsite = pair_tables(n, edges, J, eps, U, statistics)
        Hs = [G.pair_hamiltonian(n, bonds, J[r], eps[r], U[r], statistics) for r in range(R)]
    got = graph_orders(nbr, hop, onsite, dt, tol)
    want = [_rule_order(dt * float(np.abs(H.toarray()).sum(axis=1).max()), tol) for H in Hs]
    assert list(got) == want
    assert len(set(want)) >= 2
    from paper_1612_00746_amd import CtqwError
    with pytest.raises(CtqwError) as e:
        graph_orders(nbr, hop, onsite, dt, tol, max_order=min(want) - 1)
    assert e.value.status == 5


def test_graph_static_refuses_oversized_scratch_without_a_device():
    """ctqw_graph_evolve_static checks the scratch size before any device
    call: a problem needing more than CTQW_GRAPH_STATIC_BYTES is refused
    with UNSUPPORTED and a message naming the limit (runs without a GPU)."""
    from paper_1612_00746_amd import _lib as L
    lib = L.load()
    n, R = 1 << 16, 64           # 3 * n * R * 16 bytes = 192 MiB > 64 MiB
    st = lib.ctqw_graph_evolve_static(n, 0, None, None, 1, R, L.C128, 0.05, 4, 1, 1, None, None)
    assert st == L.ERR_UNSUPPORTED
    msg = lib.ctqw_last_error(None).decode()
    assert "static buffer" in msg and str(L.GRAPH_STATIC_BYTES) in msg
    # just inside the limit the size check passes and the NULL state is refused instead
    n_ok = L.GRAPH_STATIC_BYTES // (3 * 16)
    st = lib.ctqw_graph_evolve_static(n_ok, 0, None, None, 1, 1, L.C128, 0.05, 4, 1, None, None, None)
    assert st == L.ERR_INVALID_ARG
    import re
    hdr = open(HEADER).read()
    m = re.search(r"#define CTQW_GRAPH_STATIC_BYTES \((\d+)ll << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == L.GRAPH_STATIC_BYTES


def test_fermion_plans_validate_and_use_the_triangle_layout():
    """Two fermions on an open chain: accepted, stored on the triangle
    x1 <= x2 (N(N+1)/2 amplitudes, the diagonal held at 0); on a ring or
    with three particles: UNSUPPORTED; one fermion is one walker."""
    from paper_1612_00746_amd import CtqwError, Plan, make_problem
    pr, _ = make_problem(2, 3, 9, 0.05, statistics="fermion", interaction="nearest", taylor_tol=1e-12)
    p = Plan(pr)
    assert list(np.diff(p.layout())) == [45, 45, 45]
    for kw in (dict(m=2, boundary="periodic"), dict(m=3)):
        m = kw.pop("m")
        pr, _ = make_problem(m, 1, 9, 0.05, statistics="fermion", taylor_tol=1e-12, **kw)
        with pytest.raises(CtqwError) as e:
            Plan(pr)
        assert e.value.status == 2
    pr, _ = make_problem(1, 2, 9, 0.05, statistics="fermion", taylor_tol=1e-12)
    assert list(np.diff(Plan(pr).layout())) == [9, 9]


def test_three_walker_product_form_builds_for_every_order():
    """three_form = 1 factors the step's Taylor polynomial over its roots
    (the library checks that the passes' polynomials multiply back to
    sum z^k / k! to 1e-13): every order 2 .. 12 at 1, 2 and 3 terms per
    pass builds; other values of the field are rejected."""
    from paper_1612_00746_amd import CtqwError
    N = 10
    for order in range(2, 13):
        for K in (1, 2, 3):
            plan = make(m=3, R=1, n_sites=N, taylor_order=order, taylor_tol=0.0)
            plan.set_launch(terms_per_pass=K, three_form=1)
            plan.set_params(np.ones(N - 1), np.zeros(N), np.ones(1))
            assert plan.get_launch().three_form == 1
    plan = make(m=3, R=1, n_sites=N, taylor_order=6, taylor_tol=0.0)
    with pytest.raises(CtqwError):
        plan.set_launch(three_form=2)


def test_bandwidth_probe_rejects_bad_arguments_before_any_launch():
    """ctqw_bandwidth_probe validates on the host: NULL buffers, overlap,
    sizes that are not whole elements or grids, bad n, occupancy or pattern
    return INVALID_ARG without touching a device (the pointers here are
    never dereferenced)."""
    from paper_1612_00746_amd import _lib as L
    lib = L.load()
    a, b = C.c_void_p(1 << 20), C.c_void_p(1 << 30)
    bad = [
        (None, b, 1024, 0, 0, 0),
        (a, None, 1024, 0, 0, 0),
        (a, b, 0, 0, 0, 0),
        (a, C.c_void_p((1 << 20) + 512), 1024, 0, 0, 0),      # overlap
        (a, b, 1000, 0, 0, 0),                                 # not 16-byte elements
        (a, b, 3 * 128 * 128 * 8, 1, 100, 0),                  # n not a multiple of 128
        (a, b, 3 * 128 * 128 * 8 + 16, 1, 128, 0),             # not whole grids
        (a, b, 3 * 128 * 128 * 8, 1, 128, 2),                  # waves per CU below 4
        (a, b, 3 * 128 * 128 * 8, 1, 128, 33),                 # above 32
        (a, b, 1024, 2, 128, 0),                               # pattern
    ]
    for args in bad:
        assert lib.ctqw_bandwidth_probe(*args, None) == L.ERR_INVALID_ARG, args
