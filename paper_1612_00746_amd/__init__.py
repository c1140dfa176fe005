"""MI355X (gfx950) propagation of noisy many-particle quantum walks.

Python face of libctqw (include/ctqw.h).  The ``Plan`` class marshals
arguments to the C ABI and provides device memory and the HIP stream from
PyTorch; the propagation itself (stencil, Taylor series, norms,
observables) runs in the library's HIP kernels.  There is no CPU fallback:
without the built library, or without a GPU, the calls raise.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L
from ._lib import (ACC_KAHAN, ACC_PLAIN, BOSON, C64, C128, DISTINGUISHABLE, FERMION, INT_NEAREST,  # noqa: F401
                   INT_ONSITE, OBS_OCCUPATION, OBS_PAIR, OPEN, PERIODIC, RK4_ORDER, CtqwError)

__all__ = ["Plan", "CtqwError", "make_problem"]

_STAT = {"distinguishable": DISTINGUISHABLE, "boson": BOSON, "fermion": FERMION}
_BC = {"open": OPEN, "periodic": PERIODIC}
_INT = {"onsite": INT_ONSITE, "nearest": INT_NEAREST}
_DT = {"c64": C64, "c128": C128}
_ACC = {"kahan": ACC_KAHAN, "plain": ACC_PLAIN}


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def make_problem(m: int, R: int, n_sites: int | Sequence[int], dt: float, *,
                 statistics: str = "distinguishable", boundary: str = "open",
                 interaction: str = "onsite", dtype: str = "c128", accumulation: str = "kahan",
                 taylor_order: int = 0, taylor_tol: float = 0.0, taylor_max_order: int = 0,
                 renormalize: bool = False, norm_alarm: float = 0.0,
                 observables: int = OBS_OCCUPATION, method: str = "taylor"):
    """Build a ``ctqw_problem``; returns (struct, keep-alive array or None).
    method="rk4": the classical Runge-Kutta step (Alg. 2), which for this
    linear system is the degree-4 Taylor step (include/ctqw.h,
    CTQW_RK4_ORDER); taylor_order and taylor_tol must then be left unset."""
    if method == "rk4":
        if taylor_order or taylor_tol:
            raise ValueError("method='rk4' fixes the step; leave taylor_order and taylor_tol unset")
        taylor_order = RK4_ORDER
    elif method != "taylor":
        raise ValueError(f"unknown method {method!r}")
    pr = L.Problem()
    pr.m = m
    pr.statistics = _STAT[statistics]
    pr.interaction = _INT[interaction]
    pr.boundary = _BC[boundary]
    pr.dtype = _DT[dtype]
    pr.accumulation = _ACC[accumulation]
    pr.R = R
    keep = None
    if np.isscalar(n_sites):
        pr.n_sites = int(n_sites)
    else:
        keep = np.ascontiguousarray(n_sites, dtype=np.int32)
        if keep.shape[0] != R:
            raise ValueError("n_sites list must have R entries")
        pr.n_sites = 0
        pr.n_sites_per_real = _ptr(keep, C.c_int32)
    pr.dt = dt
    pr.taylor_order = taylor_order
    pr.taylor_tol = taylor_tol
    pr.taylor_max_order = taylor_max_order
    pr.renormalize = 1 if renormalize else 0
    pr.norm_alarm = norm_alarm
    pr.observables = observables
    return pr, keep


class Plan:
    """One ``ctqw_plan`` with torch-owned device buffers."""

    def __init__(self, problem: "L.Problem"):
        self.lib = L.load()
        self.problem = problem
        h = L.PlanP()
        L.check(self.lib.ctqw_plan_create(C.byref(problem), C.byref(h)))
        self.h = h
        self.R = int(problem.R)
        self.m = int(problem.m)
        self.dtype = "c128" if problem.dtype == C128 else "c64"
        if problem.n_sites > 0:
            self.Ns = [int(problem.n_sites)] * self.R
        else:
            self.Ns = [int(problem.n_sites_per_real[r]) for r in range(self.R)]
        self.periodic = problem.boundary == PERIODIC
        self._buffers = None
        self._keep = []

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.ctqw_plan_destroy(h)
            self.h = None

    def _check(self, status):
        L.check(status, self.h)

    # -------------------------------------------------------------- host side
    def set_params(self, J: np.ndarray, eps: np.ndarray, U: np.ndarray) -> None:
        J = np.ascontiguousarray(J, dtype=np.float64)
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.float64)
        self._check(self.lib.ctqw_set_params(self.h, _ptr(J, C.c_double), _ptr(eps, C.c_double),
                                             _ptr(U, C.c_double)))

    def n_bonds(self, N: int) -> int:
        return N if self.periodic else N - 1

    def get_params(self) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        """The packed J, eps, U in force (as set or drawn)."""
        J = np.zeros(sum(self.n_bonds(N) for N in self.Ns))
        eps = np.zeros(sum(self.Ns))
        U = np.zeros(self.R)
        self._check(self.lib.ctqw_get_params(self.h, _ptr(J, C.c_double), _ptr(eps, C.c_double),
                                             _ptr(U, C.c_double)))
        return J, eps, U

    def draw_params(self, *, J_base=None, eps_base=None, U_base: float = 0.0, J_noise=None, eps_noise=None,
                    U_noise=None, seed: int = 0) -> None:
        """Draw every realisation's parameters in the library (baseline plus
        a Philox4x32-10 draw per parameter).  Noises are (dist, a, b) with
        dist in {"none", "uniform", "normal"}; None means no noise."""
        dists = {"none": L.DIST_NONE, "uniform": L.DIST_UNIFORM, "normal": L.DIST_NORMAL}

        def noise(n):
            if n is None:
                return None
            d, a, b = n
            return C.byref(L.Noise(dists[d], float(a), float(b)))
        Jb = None if J_base is None else np.ascontiguousarray(J_base, dtype=np.float64)
        Eb = None if eps_base is None else np.ascontiguousarray(eps_base, dtype=np.float64)
        if Jb is not None and Jb.shape[0] < self.n_bonds(max(self.Ns)):
            raise ValueError("J_base needs n_bonds(max N) entries")
        if Eb is not None and Eb.shape[0] < max(self.Ns):
            raise ValueError("eps_base needs max N entries")
        self._check(self.lib.ctqw_draw_params(
            self.h, None if Jb is None else _ptr(Jb, C.c_double), None if Eb is None else _ptr(Eb, C.c_double),
            float(U_base), noise(J_noise), noise(eps_noise), noise(U_noise), int(seed)))

    def set_telegraph(self, amplitude: float, rate: float, seed: int = 0) -> None:
        """Switching hopping noise +-amplitude at the given rate (ctqw_set_telegraph)."""
        self._check(self.lib.ctqw_set_telegraph(self.h, float(amplitude), float(rate), int(seed)))

    def orders(self) -> np.ndarray:
        out = np.zeros(self.R, dtype=np.int32)
        self._check(self.lib.ctqw_orders(self.h, _ptr(out, C.c_int32)))
        return out

    def layout(self) -> np.ndarray:
        out = np.zeros(self.R + 1, dtype=np.int64)
        self._check(self.lib.ctqw_layout(self.h, _ptr(out, C.c_int64)))
        return out

    def sizes(self) -> tuple[int, int]:
        s, w = C.c_int64(), C.c_int64()
        self._check(self.lib.ctqw_sizes(self.h, C.byref(s), C.byref(w)))
        return s.value, w.value

    def groups(self) -> np.ndarray:
        n = C.c_int32()
        self._check(self.lib.ctqw_groups(self.h, C.byref(n), None))
        out = np.zeros(n.value, dtype=np.int32)
        self._check(self.lib.ctqw_groups(self.h, C.byref(n), _ptr(out, C.c_int32)))
        return out

    def get_launch(self) -> "L.Launch":
        l = L.Launch()
        self._check(self.lib.ctqw_get_launch(self.h, C.byref(l)))
        return l

    def set_launch(self, **kw) -> None:
        l = self.get_launch()
        for k, v in kw.items():
            setattr(l, k, int(v))
        self._check(self.lib.ctqw_set_launch(self.h, C.byref(l)))

    def work_items(self) -> tuple[int, int]:
        a, b = C.c_int64(), C.c_int64()
        self._check(self.lib.ctqw_work_items(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    # ------------------------------------------------------------ device side
    def bind(self, device: str = "cuda", stream=None) -> None:
        import torch
        state_bytes, ws_bytes = self.sizes()
        dev = torch.device(device)
        psi_a = torch.empty(max(state_bytes, 256), dtype=torch.uint8, device=dev)
        psi_b = torch.empty(max(state_bytes, 256), dtype=torch.uint8, device=dev)
        ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self._buffers = (psi_a, psi_b, ws)
        self._stream = stream
        self._check(self.lib.ctqw_bind(self.h, C.c_void_p(psi_a.data_ptr()), C.c_void_p(psi_b.data_ptr()),
                                       state_bytes, C.c_void_p(ws.data_ptr()), ws_bytes,
                                       C.c_void_p(stream.cuda_stream)))

    def init_product_state(self, sites) -> None:
        s = np.ascontiguousarray(sites, dtype=np.int32)
        per_real = 1 if s.ndim == 2 else 0
        s = s.reshape(-1)
        self._check(self.lib.ctqw_init_product_state(self.h, _ptr(s, C.c_int32), per_real))

    def state_numpy(self) -> np.ndarray:
        total = int(self.layout()[-1])
        out = np.zeros(total, dtype=np.complex128 if self.dtype == "c128" else np.complex64)
        self._check(self.lib.ctqw_get_state(self.h, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def set_state_numpy(self, psi: np.ndarray) -> None:
        psi = np.ascontiguousarray(psi, dtype=np.complex128 if self.dtype == "c128" else np.complex64)
        self._check(self.lib.ctqw_set_state(self.h, psi.ctypes.data_as(C.c_void_p), 0))

    def snapshot_len(self, obs: int) -> int:
        n = 0
        for Ng in self.groups():
            if obs & OBS_OCCUPATION:
                n += int(Ng)
            if obs & OBS_PAIR:
                n += int(Ng) * int(Ng)
        return n

    def propagate(self, n_steps: int, output_every: int = 0, obs: int = 0) -> Optional[np.ndarray]:
        if output_every > 0 and obs:
            n_out = n_steps // output_every + 1
            out = np.zeros(n_out * self.snapshot_len(obs), dtype=np.float64)
            self._check(self.lib.ctqw_propagate(self.h, n_steps, output_every, obs, _ptr(out, C.c_double)))
            return out.reshape(n_out, -1)
        self._check(self.lib.ctqw_propagate(self.h, n_steps, 0, 0, None))
        return None

    def observe(self, obs: int = OBS_OCCUPATION) -> np.ndarray:
        out = np.zeros(self.snapshot_len(obs), dtype=np.float64)
        self._check(self.lib.ctqw_observe(self.h, obs, _ptr(out, C.c_double)))
        return out

    def density_matrix(self, group: int = 0, lower_only: bool = False):
        """Ensemble-averaged density matrix of lattice-size group `group`
        (ctqw_density_matrix) as a device tensor, row-major rho[i, j]."""
        import torch
        ws_bytes = C.c_int64()
        self._check(self.lib.ctqw_density_workspace(self.h, group, C.byref(ws_bytes)))
        psi_a = self._buffers[0]
        ctype = torch.complex128 if self.dtype == "c128" else torch.complex64
        Ng = int(self.groups()[group])
        r = next(k for k, n in enumerate(self.Ns) if n == Ng)
        off = self.layout()
        D = int(off[r + 1] - off[r])          # amplitudes of one realisation of the group
        # the full matrix is written element by element; lower_only leaves the upper at zero
        alloc = torch.zeros if lower_only else torch.empty
        rho = alloc((D, D), dtype=ctype, device=psi_a.device)
        ws = torch.empty(max(ws_bytes.value, 256), dtype=torch.uint8, device=psi_a.device)
        self._check(self.lib.ctqw_density_matrix(self.h, group, C.c_void_p(rho.data_ptr()), D,
                                                 1 if lower_only else 0, C.c_void_p(ws.data_ptr()),
                                                 ws_bytes.value))
        self._stream.synchronize()
        # the buffer is column-major: its row-major view is rho transposed
        return rho.transpose(0, 1)

    def group_sizes(self, group: int) -> int:
        """Realisations in lattice-size group `group`."""
        N = int(self.groups()[group])
        return sum(1 for n in self.Ns if n == N)

    def stats(self) -> "L.StepStats":
        s = L.StepStats()
        self._check(self.lib.ctqw_stats(self.h, C.byref(s)))
        return s

    def autotune(self, cache_path: Optional[str] = None, steps: int = 3) -> tuple["L.Launch", float]:
        """Time the launch shapes and apply the fastest (overwrites the state)."""
        best, ms = L.Launch(), C.c_double()
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.ctqw_autotune(self.h, path, steps, C.byref(best), C.byref(ms)))
        return best, ms.value

    # ------------------------------------------------------------ gradients
    def _grad_workspace(self, n_steps: int, ckpt_every: int):
        import torch
        b = C.c_int64()
        self._check(self.lib.ctqw_gradient_workspace(self.h, n_steps, ckpt_every, C.byref(b)))
        ws = getattr(self, "_grad_ws", None)
        if ws is None or ws.numel() < b.value:
            self._grad_ws = None
            ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=self._buffers[0].device)
            self._grad_ws = ws
        return ws, b.value

    def forward_ckpt(self, n_steps: int, ckpt_every: int) -> None:
        ws, nb = self._grad_workspace(n_steps, ckpt_every)
        self._check(self.lib.ctqw_forward_ckpt(self.h, n_steps, ckpt_every, C.c_void_p(ws.data_ptr()), ws.numel()))

    def backward(self, site_weights, kind: str = "product"):
        """(loss, dL/dJbar [n_bonds], dL/depsbar [N]) after forward_ckpt."""
        g = np.ascontiguousarray(site_weights, dtype=np.float64)
        N = g.shape[0]
        nb = N if self.problem.boundary == PERIODIC else N - 1
        gJ = np.zeros(nb)
        gE = np.zeros(N)
        loss = C.c_double()
        ws = self._grad_ws
        k = L.LOSS_PRODUCT if kind == "product" else L.LOSS_ONE_BODY
        self._check(self.lib.ctqw_backward(self.h, k, _ptr(g, C.c_double), C.c_void_p(ws.data_ptr()), ws.numel(),
                                           C.byref(loss), _ptr(gJ, C.c_double), _ptr(gE, C.c_double)))
        return loss.value, gJ, gE

    def loss(self, site_weights, kind: str = "product") -> float:
        """The ensemble loss at the current state (needs forward_ckpt's workspace)."""
        g = np.ascontiguousarray(site_weights, dtype=np.float64)
        ws = getattr(self, "_grad_ws", None)
        if ws is None:
            ws, _ = self._grad_workspace(0, 1)
        out = C.c_double()
        k = L.LOSS_PRODUCT if kind == "product" else L.LOSS_ONE_BODY
        self._check(self.lib.ctqw_loss(self.h, k, _ptr(g, C.c_double), C.c_void_p(ws.data_ptr()), ws.numel(),
                                       C.byref(out)))
        return out.value

    def gradient(self, n_steps: int, ckpt_every: int, site_weights, kind: str = "product"):
        self.forward_ckpt(n_steps, ckpt_every)
        return self.backward(site_weights, kind)

    def set_timing(self, enable: bool) -> None:
        self._check(self.lib.ctqw_set_timing(self.h, 1 if enable else 0))

    def get_timing(self) -> tuple[float, int]:
        ms, n = C.c_double(), C.c_int64()
        self._check(self.lib.ctqw_get_timing(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def realization_norms(self) -> tuple[np.ndarray, np.ndarray]:
        n2 = np.zeros(self.R)
        t2 = np.zeros(self.R)
        self._check(self.lib.ctqw_realization_norms(self.h, _ptr(n2, C.c_double), _ptr(t2, C.c_double)))
        return n2, t2


# ------------------------------------------------------------------ graphs
def lattice_edges(shape: Sequence[int], periodic: bool = False) -> np.ndarray:
    """Bonds of a q-dimensional regular lattice with nearest-neighbour
    coupling along each axis (Sec. 2, k_i = 1), nodes numbered row-major
    (last axis fastest).  Returns int32 [E, 2] with a < b in each pair; a
    periodic axis of length > 2 adds the wrap-around bond."""
    shape = [int(s) for s in shape]
    if not shape or min(shape) < 1:
        raise ValueError("lattice sides must be positive")
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    out = []
    for ax, s in enumerate(shape):
        if s < 2:
            continue
        a = np.take(idx, np.arange(s - 1), axis=ax).ravel()
        b = np.take(idx, np.arange(1, s), axis=ax).ravel()
        out.append(np.stack([a, b], 1))
        if periodic and s > 2:
            a = np.take(idx, [s - 1], axis=ax).ravel()
            b = np.take(idx, [0], axis=ax).ravel()
            out.append(np.stack([np.minimum(a, b), np.maximum(a, b)], 1))
    if not out:
        return np.zeros((0, 2), dtype=np.int32)
    return np.concatenate(out).astype(np.int32)


def graph_tables(n_nodes: int, edges: np.ndarray, J: np.ndarray, eps: Optional[np.ndarray] = None,
                 U: Optional[np.ndarray] = None, m: int = 1,
                 statistics: str = "distinguishable") -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """ctqw_graph_tables: the ELL tables of ctqw_graph_evolve for m = 1 or
    2 particles on the graph with the undirected bonds `edges` (int [E, 2]),
    built by the library from J [R, E], eps [R, n] (zeros if None) and, for
    two particles, U [R] and the statistics.  Returns nbr int32 [width,
    states], hop float64 [R, width, states] and onsite float64 [R, states]."""
    lib = L.load()
    edges = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).reshape(-1, 2), dtype=np.int32)
    J = np.ascontiguousarray(np.atleast_2d(np.asarray(J, dtype=np.float64)))
    R = J.shape[0]
    if J.shape[1] != len(edges):
        raise ValueError("J must be [R, E]")
    eps = np.zeros((R, n_nodes)) if eps is None else np.asarray(eps, dtype=np.float64)
    eps = np.ascontiguousarray(np.atleast_2d(eps))
    if eps.shape != (R, n_nodes):
        raise ValueError("eps must be [R, n]")
    if m == 2:
        U = np.ascontiguousarray(np.atleast_1d(np.asarray(U, dtype=np.float64)))
        if U.shape != (R,):
            raise ValueError("U must be [R]")
    ns, w = C.c_int32(), C.c_int32()
    p = lambda a: C.c_void_p(a.ctypes.data) if a is not None and a.size else None  # noqa: E731
    stat = _STAT[statistics]
    L.check(lib.ctqw_graph_tables(int(n_nodes), len(edges), p(edges), int(m), stat, R, None, None, None,
                                  C.byref(ns), C.byref(w), None, None, None))
    D, W = ns.value, w.value
    nbr = np.full((W, D), -1, dtype=np.int32)
    hop = np.zeros((R, W, D))
    onsite = np.zeros((R, D))
    L.check(lib.ctqw_graph_tables(int(n_nodes), len(edges), p(edges), int(m), stat, R, p(J), p(eps),
                                  p(U) if m == 2 else None, C.byref(ns), C.byref(w), C.c_void_p(nbr.ctypes.data),
                                  C.c_void_p(hop.ctypes.data), C.c_void_p(onsite.ctypes.data)))
    return nbr, hop, onsite


def ell_tables(n_nodes: int, edges: np.ndarray, J: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """One particle: nbr int32 [width, n] and hop float64 [R, width, n] of
    ctqw_graph_tables for the bond list `edges` and couplings J [R, E]."""
    nbr, hop, _ = graph_tables(n_nodes, edges, J)
    return nbr, hop


def pair_tables(n_nodes: int, edges: np.ndarray, J: np.ndarray, eps: np.ndarray, U: np.ndarray,
                statistics: str = "distinguishable") -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Two particles on a graph as one particle on the pair graph:
    ctqw_graph_tables with m = 2 (J [R, E], eps [R, n], U [R]).  Returns
    nbr int32 [2 width, D], hop float64 [R, 2 width, D] and onsite float64
    [R, D]."""
    return graph_tables(n_nodes, edges, J, eps, U, m=2, statistics=statistics)


def _graph_args(nbr, hop, onsite, psi, n_steps, norms):
    """Check the device tensors of graph_evolve(_static); returns (R, n,
    width, dtype)."""
    import torch
    R, n = psi.shape
    width = nbr.shape[0]
    if psi.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("psi must be complex64 or complex128")
    c128 = psi.dtype == torch.complex128
    real = torch.float64 if c128 else torch.float32
    for t, dt_, shp in ((nbr, torch.int32, (width, n)), (hop, real, (R, width, n)), (onsite, real, (R, n)),
                        (psi, psi.dtype, (R, n))):
        if t.dtype != dt_ or tuple(t.shape) != shp or not t.is_contiguous() or t.device != psi.device:
            raise ValueError(f"expected a contiguous {dt_} tensor of shape {shp} on {psi.device}")
    if norms is not None and (norms.dtype != torch.float64 or tuple(norms.shape) != (int(n_steps), R)
                              or not norms.is_contiguous() or norms.device != psi.device):
        raise ValueError(f"norms must be a contiguous float64 tensor of shape ({n_steps}, {R}) on {psi.device}")
    return R, n, width, (C128 if c128 else C64)


def graph_evolve(nbr, hop, onsite, psi, dt: float, order: int, n_steps: int, workspace=None, norms=None) -> None:
    """ctqw_graph_evolve on device tensors: one particle on a general graph,
    R realisations advanced in place.  nbr int32 [width, n]; psi complex128
    [R, n] with hop float64 [R, width, n] and onsite float64 [R, n], or
    psi complex64 with float32 tables; all contiguous on one device.  norms
    (optional) float64 [n_steps, R] receives each step's squared norms.
    Enqueued on that device's current stream."""
    import torch
    lib = L.load()
    R, n, width, dtype = _graph_args(nbr, hop, onsite, psi, n_steps, norms)
    b = C.c_int64()
    L.check(lib.ctqw_graph_workspace(n, R, dtype, C.byref(b)))
    if workspace is None:
        workspace = torch.empty(b.value, dtype=torch.uint8, device=psi.device)
    stream = torch.cuda.current_stream(psi.device).cuda_stream
    p = lambda t: C.c_void_p(t.data_ptr()) if t.numel() else None  # noqa: E731
    L.check(lib.ctqw_graph_evolve(n, width, p(nbr), p(hop), p(onsite), R, dtype, float(dt), int(order), int(n_steps),
                                  p(psi), p(workspace), workspace.numel() * workspace.element_size(),
                                  p(norms) if norms is not None else None, C.c_void_p(stream)))


def graph_evolve_static(nbr, hop, onsite, psi, dt: float, order: int, n_steps: int, norms=None) -> None:
    """ctqw_graph_evolve_static: graph_evolve without a workspace, the
    library's fixed device array (GRAPH_STATIC_BYTES per device) taking its
    place, for callers that cannot allocate.  Calls that overlap on one
    device race on that array."""
    import torch
    lib = L.load()
    R, n, width, dtype = _graph_args(nbr, hop, onsite, psi, n_steps, norms)
    stream = torch.cuda.current_stream(psi.device).cuda_stream
    p = lambda t: C.c_void_p(t.data_ptr()) if t.numel() else None  # noqa: E731
    L.check(lib.ctqw_graph_evolve_static(n, width, p(nbr), p(hop), p(onsite), R, dtype, float(dt), int(order),
                                         int(n_steps), p(psi), p(norms) if norms is not None else None,
                                         C.c_void_p(stream)))


def bandwidth_probe(src, dst, pattern: int, n: int = 1024, waves_per_cu: int = 0) -> None:
    """ctqw_bandwidth_probe on two contiguous, non-overlapping device tensors
    of the same byte size: pattern 0 copies src to dst flat, pattern 1 with
    the step kernel's band row sweep over n x n complex64 grids (measurement
    only).  Enqueued on the device's current stream."""
    import torch
    lib = L.load()
    nbytes = src.numel() * src.element_size()
    if (not src.is_contiguous() or not dst.is_contiguous() or dst.numel() * dst.element_size() != nbytes
            or src.device != dst.device or src.device.type != "cuda"):
        raise ValueError("src and dst must be contiguous device tensors of the same size on one device")
    stream = torch.cuda.current_stream(src.device).cuda_stream
    L.check(lib.ctqw_bandwidth_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, int(pattern),
                                     int(n), int(waves_per_cu), C.c_void_p(stream)))


def lattice_evolve(Jx, Jy, eps, psi, dt: float, order: int, n_steps: int, periodic=(False, False),
                   workspace=None, norms=None) -> None:
    """ctqw_lattice_evolve on device tensors: one particle on an Lx x Ly
    lattice, R realisations advanced in place with all `order` terms of a
    step in one pass.  psi complex64 [R, Ly, Lx] with Jx, Jy, eps float32
    [R, Ly, Lx] (or complex128 with float64 tables); Jx[r, y, x] couples
    (x, y) to (x + 1, y), Jy[r, y, x] couples (x, y) to (x, y + 1).
    periodic = (x ring, y ring).  norms (optional) float64 [n_steps, R].
    Enqueued on the device's current stream."""
    import torch
    lib = L.load()
    if psi.dtype not in (torch.complex64, torch.complex128) or psi.dim() != 3:
        raise ValueError("psi must be a complex64 or complex128 tensor of shape (R, Ly, Lx)")
    R, Ly, Lx = psi.shape
    c128 = psi.dtype == torch.complex128
    real = torch.float64 if c128 else torch.float32
    for t in (Jx, Jy, eps, psi):
        if t.dtype not in (real, psi.dtype) or tuple(t.shape) != (R, Ly, Lx) or not t.is_contiguous() \
                or t.device != psi.device:
            raise ValueError(f"expected contiguous tensors of shape {(R, Ly, Lx)} on {psi.device}")
    for t in (Jx, Jy, eps):
        if t.dtype != real:
            raise ValueError(f"tables must be {real}")
    if norms is not None and (norms.dtype != torch.float64 or tuple(norms.shape) != (int(n_steps), R)
                              or not norms.is_contiguous() or norms.device != psi.device):
        raise ValueError(f"norms must be a contiguous float64 tensor of shape ({n_steps}, {R}) on {psi.device}")
    dtype = C128 if c128 else C64
    px, py = int(bool(periodic[0])), int(bool(periodic[1]))
    b = C.c_int64()
    L.check(lib.ctqw_lattice_workspace(Lx, Ly, R, dtype, int(order), px, C.byref(b)))
    if workspace is None:
        workspace = torch.empty(b.value, dtype=torch.uint8, device=psi.device)
    stream = torch.cuda.current_stream(psi.device).cuda_stream
    p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    L.check(lib.ctqw_lattice_evolve(Lx, Ly, px, py, R, p(Jx), p(Jy), p(eps), dtype, float(dt), int(order),
                                    int(n_steps), p(psi), p(workspace), workspace.numel() * workspace.element_size(),
                                    p(norms) if norms is not None else None, C.c_void_p(stream)))


def graph_orders(nbr: np.ndarray, hop: np.ndarray, onsite: np.ndarray, dt: float, tol: float,
                 max_order: int = 64) -> np.ndarray:
    """ctqw_graph_orders on host tables (the layouts of graph_evolve, FP64):
    each realisation's a-priori Taylor order for the tolerance tol."""
    lib = L.load()
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    hop = np.ascontiguousarray(hop, dtype=np.float64)
    onsite = np.ascontiguousarray(np.atleast_2d(onsite), dtype=np.float64)
    R, n = onsite.shape
    width = nbr.shape[0]
    if nbr.shape != (width, n) or hop.shape != (R, width, n):
        raise ValueError("tables must be nbr [width, n], hop [R, width, n], onsite [R, n]")
    out = np.zeros(R, dtype=np.int32)
    p = lambda a: C.c_void_p(a.ctypes.data) if a.size else None  # noqa: E731
    L.check(lib.ctqw_graph_orders(n, width, p(nbr), p(hop), p(onsite), R, float(dt), float(tol), int(max_order),
                                  C.c_void_p(out.ctypes.data)))
    return out
