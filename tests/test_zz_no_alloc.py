"""GPU check of ctqw_graph_evolve_static, the entry point that allocates
nothing: its output must equal ctqw_graph_evolve's (same kernels, the
library's fixed device array in place of the caller's workspace) bit for
bit, on two calls in a row, the second with a smaller input (the array
keeps the first call's contents, which must not leak into the second), in
complex128 and complex64, with the per-step norms; and the entry point
refuses a problem whose scratch exceeds the array before touching the
device."""

import numpy as np
import pytest

from oracle import graph as G

from _helpers import say

pytestmark = pytest.mark.gpu


def tables(shape, R, seed, c64):
    import torch
    from paper_1612_00746_amd import ell_tables
    n = int(np.prod(shape))
    edges = np.array(G.lattice_bonds(shape, False), dtype=np.int64).reshape(-1, 2)
    g = np.random.default_rng(seed)
    J = 1.0 + 0.1 * g.standard_normal((R, len(edges)))
    eps = g.uniform(-0.5, 0.5, (R, n))
    nbr, hop = ell_tables(n, edges, J)
    psi = g.standard_normal((R, n)) + 1j * g.standard_normal((R, n))
    psi /= np.linalg.norm(psi, axis=1, keepdims=True)
    rt = np.float32 if c64 else np.float64
    ct = np.complex64 if c64 else np.complex128
    dev = "cuda"
    return (torch.from_numpy(nbr).to(dev), torch.from_numpy(np.ascontiguousarray(hop, dtype=rt)).to(dev),
            torch.from_numpy(np.ascontiguousarray(eps, dtype=rt)).to(dev), torch.from_numpy(psi.astype(ct)).to(dev))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_static_scratch_matches_workspace_entry(dtype):
    import torch
    from paper_1612_00746_amd import graph_evolve, graph_evolve_static
    c64 = dtype == "c64"
    # first call large, second smaller: (shape, R, order, steps)
    for k, (shape, R, order, steps) in enumerate([((24, 21), 96, 9, 5), ((7, 5), 9, 6, 4), ((6, 4), 3, 1, 3)]):
        say(f"case: static scratch {dtype} call {k}: lattice {shape}, R={R}, order {order}, steps {steps}")
        nbr, hop, eps, psi = tables(shape, R, 100 + k, c64)
        a = psi.clone()
        b = psi.clone()
        na = torch.full((steps, R), -1.0, dtype=torch.float64, device="cuda")
        nb = torch.full((steps, R), -2.0, dtype=torch.float64, device="cuda")
        graph_evolve(nbr, hop, eps, a, 0.05, order, steps, norms=na)
        graph_evolve_static(nbr, hop, eps, b, 0.05, order, steps, norms=nb)
        torch.cuda.synchronize()
        assert torch.equal(a, b), float((a - b).abs().max())
        assert torch.equal(na, nb)
        assert not torch.equal(a, psi)     # the state moved


def test_static_scratch_refuses_oversized_problems():
    import torch
    from paper_1612_00746_amd import _lib as L
    from paper_1612_00746_amd import graph_evolve_static
    nbr, hop, eps, psi = tables((4, 4), 2, 7, False)
    lib = L.load()
    # 3 * n * R * 16 bytes > 64 MiB: refused with UNSUPPORTED before any device work
    n, R = 1 << 16, 64
    st = lib.ctqw_graph_evolve_static(n, 0, None, None, 1, R, L.C128, 0.05, 4, 1, 1, None, None)
    assert st == L.ERR_UNSUPPORTED
    assert b"static buffer" in lib.ctqw_last_error(None)
    before = psi.clone()
    graph_evolve_static(nbr, hop, eps, psi, 0.05, 4, 0)   # zero steps: state unchanged
    torch.cuda.synchronize()
    assert torch.equal(before, psi)
