"""ctypes declarations of the C ABI in include/ctqw.h (argument marshalling
only; every step of the propagation runs in libctqw's HIP kernels).

The library is loaded from ``libctqw.so`` next to this file; importing
fails loudly if it has not been built (``python -c "import __graft_entry__
as g; g.build()"`` or ``python paper_1612_00746_amd/build.py``).
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctqw.so")

# enums / flags (mirror include/ctqw.h)
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NOT_CONVERGED, \
    ERR_NUMERICAL, ERR_STATE = range(8)
DISTINGUISHABLE, BOSON, FERMION = 0, 1, 2
OPEN, PERIODIC = 0, 1
INT_ONSITE, INT_NEAREST = 0, 1
C64, C128 = 0, 1
ACC_KAHAN, ACC_PLAIN = 0, 1
OBS_OCCUPATION, OBS_PAIR = 1, 2
LOSS_ONE_BODY, LOSS_PRODUCT = 0, 1
DIST_NONE, DIST_UNIFORM, DIST_NORMAL = 0, 1, 2
RK4_ORDER = 4
GRAPH_STATIC_BYTES = 64 << 20


class Problem(C.Structure):
    _fields_ = [
        ("m", C.c_int32),
        ("statistics", C.c_int32),
        ("interaction", C.c_int32),
        ("boundary", C.c_int32),
        ("dtype", C.c_int32),
        ("accumulation", C.c_int32),
        ("R", C.c_int64),
        ("n_sites", C.c_int32),
        ("n_sites_per_real", C.POINTER(C.c_int32)),
        ("dt", C.c_double),
        ("taylor_order", C.c_int32),
        ("taylor_tol", C.c_double),
        ("taylor_max_order", C.c_int32),
        ("renormalize", C.c_int32),
        ("norm_alarm", C.c_double),
        ("observables", C.c_uint32),
    ]


class Noise(C.Structure):
    _fields_ = [("dist", C.c_int32), ("a", C.c_double), ("b", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [
        ("steps_done", C.c_int64),
        ("min_norm", C.c_double),
        ("max_norm", C.c_double),
        ("max_tail_ratio", C.c_double),
        ("min_order", C.c_int32),
        ("max_order", C.c_int32),
        ("alarms", C.c_int64),
        ("flags", C.c_int32),
    ]


class Launch(C.Structure):
    _fields_ = [
        ("cols_per_lane", C.c_int32),
        ("waves_per_block", C.c_int32),
        ("persistent", C.c_int32),
        ("use_graph", C.c_int32),
        ("waves_per_cu", C.c_int32),
        ("chunked", C.c_int32),
        ("band_align", C.c_int32),
        ("terms_per_pass", C.c_int32),
        ("band_mode", C.c_int32),
        ("three_form", C.c_int32),
        ("row_segments", C.c_int32),
    ]


PlanP = C.c_void_p
dp = C.POINTER(C.c_double)
i32p = C.POINTER(C.c_int32)
i64p = C.POINTER(C.c_int64)

# name -> (restype, argtypes); every entry point declared in include/ctqw.h
SIGNATURES = {
    "ctqw_plan_create": (C.c_int, [C.POINTER(Problem), C.POINTER(PlanP)]),
    "ctqw_plan_destroy": (C.c_int, [PlanP]),
    "ctqw_set_params": (C.c_int, [PlanP, dp, dp, dp]),
    "ctqw_get_params": (C.c_int, [PlanP, dp, dp, dp]),
    "ctqw_draw_params": (C.c_int, [PlanP, dp, dp, C.c_double, C.POINTER(Noise), C.POINTER(Noise),
                                   C.POINTER(Noise), C.c_uint64]),
    "ctqw_orders": (C.c_int, [PlanP, i32p]),
    "ctqw_layout": (C.c_int, [PlanP, i64p]),
    "ctqw_sizes": (C.c_int, [PlanP, i64p, i64p]),
    "ctqw_bind": (C.c_int, [PlanP, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "ctqw_init_product_state": (C.c_int, [PlanP, i32p, C.c_int32]),
    "ctqw_set_state": (C.c_int, [PlanP, C.c_void_p, C.c_int32]),
    "ctqw_get_state": (C.c_int, [PlanP, C.c_void_p, C.c_int32]),
    "ctqw_propagate": (C.c_int, [PlanP, C.c_int64, C.c_int64, C.c_uint32, dp]),
    "ctqw_observe": (C.c_int, [PlanP, C.c_uint32, dp]),
    "ctqw_groups": (C.c_int, [PlanP, i32p, i32p]),
    "ctqw_density_workspace": (C.c_int, [PlanP, C.c_int32, i64p]),
    "ctqw_set_telegraph": (C.c_int, [PlanP, C.c_double, C.c_double, C.c_uint64]),
    "ctqw_density_matrix": (C.c_int, [PlanP, C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int64]),
    "ctqw_graph_orders": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                    C.c_double, C.c_int32, C.c_void_p]),
    "ctqw_graph_workspace": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, i64p]),
    "ctqw_graph_tables": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, i32p, i32p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ctqw_graph_evolve": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                    C.c_double, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_void_p]),
    "ctqw_graph_evolve_static": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                           C.c_int32, C.c_double, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "ctqw_lattice_workspace": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, i64p]),
    "ctqw_lattice_evolve": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_int64, C.c_void_p,
                                      C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ctqw_stats": (C.c_int, [PlanP, C.POINTER(StepStats)]),
    "ctqw_realization_norms": (C.c_int, [PlanP, dp, dp]),
    "ctqw_get_launch": (C.c_int, [PlanP, C.POINTER(Launch)]),
    "ctqw_set_launch": (C.c_int, [PlanP, C.POINTER(Launch)]),
    "ctqw_work_items": (C.c_int, [PlanP, i64p, i64p]),
    "ctqw_autotune": (C.c_int, [PlanP, C.c_char_p, C.c_int32, C.POINTER(Launch), dp]),
    "ctqw_gradient_workspace": (C.c_int, [PlanP, C.c_int64, C.c_int64, i64p]),
    "ctqw_gradient": (C.c_int, [PlanP, C.c_int64, C.c_int64, C.c_int32, dp, C.c_void_p, C.c_int64, dp, dp, dp]),
    "ctqw_forward_ckpt": (C.c_int, [PlanP, C.c_int64, C.c_int64, C.c_void_p, C.c_int64]),
    "ctqw_backward": (C.c_int, [PlanP, C.c_int32, dp, C.c_void_p, C.c_int64, dp, dp, dp]),
    "ctqw_loss": (C.c_int, [PlanP, C.c_int32, dp, C.c_void_p, C.c_int64, dp]),
    "ctqw_set_timing": (C.c_int, [PlanP, C.c_int32]),
    "ctqw_get_timing": (C.c_int, [PlanP, dp, i64p]),
    "ctqw_bandwidth_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_void_p]),
    "ctqw_status_string": (C.c_char_p, [C.c_int]),
    "ctqw_last_error": (C.c_char_p, [PlanP]),
    "ctqw_version": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libctqw.so is not built ({path}); run paper_1612_00746_amd/build.py")
    # PyTorch ships its own HIP runtime under the same soname.  Loading it
    # first makes libctqw resolve to that runtime, so torch's device memory
    # and streams and libctqw's kernels share one HIP context.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class CtqwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} [status {status}]")
        self.status = status


def check(status: int, plan=None) -> None:
    if status != OK:
        lib = load()
        msg = lib.ctqw_last_error(plan).decode() or lib.ctqw_status_string(status).decode()
        raise CtqwError(status, msg)
