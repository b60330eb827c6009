"""ctypes declarations for libfsp.so (the C ABI of include/fsp.h).

Loading fails loudly: there is no fallback implementation of any call.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_size_t, c_uint, c_void_p
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsp.so")

FSP_OK = 0
FSP_ERR_INVALID_ARG = 1
FSP_ERR_UNSUPPORTED_SIZE = 2
FSP_ERR_BOX_ASPECT = 3
FSP_ERR_OUT_OF_MEMORY = 4
FSP_ERR_NOT_READY = 5
FSP_ERR_DEVICE = 6

GREENS = {"hockney": 0, "vico": 1, "vico_dct": 2}
NUM_VARIANTS = 3
FUSED = 3  # schedule value of passes 1-3 selecting the fused small-grid kernel
PLANE = 4  # schedule value of passes 0-1 (both) or 3-4 (both) selecting the plane kernels
FSP_WANT_GRAD = 1  # plan flag: derivative tables and a workspace for fsp_solve_grad
FSP_PERIODIC = (2, 4, 8)  # plan flags: axis 0, 1, 2 periodic
PREC = {"f32": 0, "f64": 1}

# every symbol include/fsp.h declares
EXPORTS = (
    "fsp_plan_create", "fsp_plan_bytes", "fsp_plan_precompute_bytes", "fsp_plan_bind",
    "fsp_plan_share_ghat", "fsp_precompute", "fsp_solve", "fsp_solve_passes", "fsp_solve_batched", "fsp_plan_destroy",
    "fsp_plan_ghat_layout", "fsp_plan_model_bytes", "fsp_status_str", "fsp_last_error", "fsp_version",
    "fsp_batch_create", "fsp_batch_launch", "fsp_batch_destroy", "fsp_batch_set_io",
    "fsp_plan_get_schedule", "fsp_plan_set_schedule", "fsp_autotune", "fsp_autotune_batch",
    "fsp_solve_grad", "fsp_plan_octant_offset", "fsp_solve_static",
)

# every symbol include/fsp_serve.h declares
SERVE_EXPORTS = ("fsp_server_create", "fsp_server_run", "fsp_server_get_stats", "fsp_server_destroy")

# size of the library's static workspace used by fsp_solve_static (FSP_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 80 * 1024 * 1024


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", c_int * 3),
        ("lo", c_double * 3),
        ("hi", c_double * 3),
        ("greens", c_int),
        ("prec", c_int),
        ("alpha", c_double),
        ("g0", c_double),
        ("flags", c_uint),
    ]


class Request(ctypes.Structure):
    """fsp_request (include/fsp_serve.h)."""
    _fields_ = [
        ("t_arrival", c_double),
        ("n", c_int * 3),
        ("greens", c_int),
        ("prec", c_int),
        ("lo", c_double * 3),
        ("hi", c_double * 3),
        ("alpha", c_double),
        ("rho", c_void_p),
        ("phi", c_void_p),
    ]


class RequestResult(ctypes.Structure):
    """fsp_request_result (include/fsp_serve.h)."""
    _fields_ = [
        ("t_arrival", c_double),
        ("t_admit", c_double),
        ("t_done", c_double),
        ("t_seen", c_double),
        ("refresh_ms", ctypes.c_float),
        ("status", c_int),
        ("slot", c_int),
        ("launch_size", c_int),
    ]


class ServerStats(ctypes.Structure):
    """fsp_server_stats (include/fsp_serve.h)."""
    _fields_ = [
        ("budget_bytes", c_size_t),
        ("peak_held_bytes", c_size_t),
        ("held_bytes", c_size_t),
        ("launches", ctypes.c_longlong),
        ("refreshes", ctypes.c_longlong),
        ("evictions", ctypes.c_longlong),
        ("rejected", ctypes.c_longlong),
        ("refresh_ms_total", c_double),
    ]


class FspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


_lib = None


def load(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libfsp.so (built by ``python -m paper_2405_02603_amd.build``).

    ``FSP_LIBRARY`` names another build of the same library to load instead.
    """
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("FSP_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"libfsp.so not found at {path}; build it with "
                          "`python -m paper_2405_02603_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "fsp_plan_create": (c_int, [POINTER(PlanDesc), POINTER(c_void_p)]),
        "fsp_plan_bytes": (c_int, [P, POINTER(c_size_t), POINTER(c_size_t)]),
        "fsp_plan_precompute_bytes": (c_int, [P, POINTER(c_size_t)]),
        "fsp_plan_bind": (c_int, [P, P, P]),
        "fsp_plan_share_ghat": (c_int, [P, P]),
        "fsp_precompute": (c_int, [P, P]),
        "fsp_solve": (c_int, [P, P, P, P]),
        "fsp_solve_static": (c_int, [P, P, P, P]),
        "fsp_solve_passes": (c_int, [P, P, P, c_int, c_int, P]),
        "fsp_solve_batched": (c_int, [c_int, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p), P]),
        "fsp_plan_destroy": (c_int, [P]),
        "fsp_batch_create": (c_int, [c_int, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                     POINTER(c_void_p)]),
        "fsp_batch_launch": (c_int, [P, P]),
        "fsp_batch_set_io": (c_int, [P, POINTER(c_void_p), POINTER(c_void_p), P]),
        "fsp_plan_get_schedule": (c_int, [P, POINTER(c_int)]),
        "fsp_plan_set_schedule": (c_int, [P, POINTER(c_int)]),
        "fsp_autotune": (c_int, [P, P, P, c_int, P, POINTER(ctypes.c_float)]),
        "fsp_autotune_batch": (c_int, [c_int, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p), c_int, P]),
        "fsp_batch_destroy": (c_int, [P]),
        "fsp_plan_ghat_layout": (c_int, [P, POINTER(c_size_t), POINTER(c_int)]),
        "fsp_plan_model_bytes": (c_int, [P, POINTER(c_double)]),
        "fsp_solve_grad": (c_int, [P, P, P, P, P]),
        "fsp_plan_octant_offset": (c_int, [P, c_int, POINTER(c_size_t)]),
        "fsp_server_create": (c_int, [c_size_t, c_int, c_int, POINTER(c_void_p)]),
        "fsp_server_run": (c_int, [P, c_int, POINTER(Request), POINTER(RequestResult), c_double, c_double]),
        "fsp_server_get_stats": (c_int, [P, POINTER(ServerStats)]),
        "fsp_server_destroy": (c_int, [P]),
        "fsp_status_str": (c_char_p, [c_int]),
        "fsp_last_error": (c_char_p, []),
        "fsp_version": (c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str = "") -> None:
    if status != FSP_OK:
        lib = load()
        name = lib.fsp_status_str(status).decode()
        detail = lib.fsp_last_error().decode()
        raise FspError(status, f"{what}: {name}: {detail}" if what else f"{name}: {detail}")
