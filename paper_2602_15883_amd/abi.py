"""ctypes declarations of the C ABI in include/ddpinn.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t,
                    c_uint8, c_uint32, c_void_p)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddpinn.so")

PINN_OK = 0
PINN_E_INVAL = -1
PINN_E_NOMEM = -2
PINN_E_DEVICE = -3
PINN_E_BUDGET = -4
PINN_E_NONFINITE = -5
PINN_E_UNSUPPORTED = -6
STATUS_NAMES = {0: "PINN_OK", -1: "PINN_E_INVAL", -2: "PINN_E_NOMEM", -3: "PINN_E_DEVICE",
                -4: "PINN_E_BUDGET", -5: "PINN_E_NONFINITE", -6: "PINN_E_UNSUPPORTED"}

PINN_GRAPH = 1
PINN_NO_UPDATE = 1
PINN_CHECK_FINITE = 2
PINN_PER_SUBDOMAIN = 4
PINN_TIME_KERNEL = 8
PINN_Q_VALUE = 0
PINN_Q_UVPW = 1
PINN_Q_CHANNELS = 2
PINN_Q_RESIDUAL = 3

# every symbol include/ddpinn.h declares
EXPORTS = ("pinn_num_params", "pinn_create", "pinn_step", "pinn_query_scratch_bytes",
           "pinn_query", "pinn_query_noalloc", "pinn_exchange", "pinn_refresh", "pinn_destroy",
           "pinn_get_launch_info", "pinn_last_error", "pinn_kernel_time",
           "pinn_evaluate_scratch_bytes", "pinn_evaluate", "pinn_check_guards")


class PinnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class PinnConfig(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("width", c_int32), ("depth", c_int32), ("n_sub", c_int32),
                ("activation", c_int32), ("flags", c_uint32), ("nu", c_double),
                ("lam", c_float * 6), ("lr", c_float), ("beta1", c_float), ("beta2", c_float),
                ("eps", c_float), ("tile_points", c_int32), ("blocks_per_cu", c_int32),
                ("max_query_points", c_int64), ("comp_w", c_float * 3), ("clip_norm", c_float),
                ("lr_factor", c_float), ("lr_interval", c_int32), ("gemm_priority_off", c_int32),
                ("ranges_per_wg", c_int32), ("guard_bytes", c_int32)]


class PinnSubdomain(ctypes.Structure):
    _fields_ = [("lo", c_float * 4), ("hi", c_float * 4), ("is_master", c_int32),
                ("theta", c_void_p), ("adam_m", c_void_p), ("adam_v", c_void_p),
                ("pde_x", c_void_p), ("n_pde", c_int64),
                ("obs_x", c_void_p), ("obs_u", c_void_p), ("n_obs", c_int64),
                ("gh_x", c_void_p), ("gh_up", c_void_p), ("gh_kind", c_void_p), ("n_gh", c_int64),
                ("anc_x", c_void_p), ("anc_p", c_void_p), ("n_anc", c_int64)]


class PinnFace(ctypes.Structure):
    _fields_ = [("a", c_int32), ("b", c_int32), ("first", c_int64), ("count", c_int64)]


class PinnLaunchInfo(ctypes.Structure):
    _fields_ = [("tile_points", c_int32), ("value_points", c_int32), ("n_wg", c_int32),
                ("n_items", c_int32), ("n_segments", c_int32), ("threads", c_int32),
                ("lds_bytes", c_int64), ("stash_bytes", c_int64), ("slab_floats", c_int64)]


_lib = None


def lib():
    """Load libddpinn.so.  Raises if it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950) first")
    L = ctypes.CDLL(LIB_PATH)
    L.pinn_num_params.restype = c_int64
    L.pinn_num_params.argtypes = [c_int32, c_int32, c_int32]
    L.pinn_create.restype = c_int32
    L.pinn_create.argtypes = [POINTER(PinnConfig), POINTER(PinnSubdomain), c_void_p,
                              POINTER(c_size_t), c_void_p, POINTER(c_void_p)]
    L.pinn_step.restype = c_int32
    L.pinn_step.argtypes = [c_void_p, c_int64, c_uint32, c_void_p, c_void_p, c_void_p]
    L.pinn_query_scratch_bytes.restype = c_size_t
    L.pinn_query_scratch_bytes.argtypes = [c_void_p, c_int64]
    L.pinn_query.restype = c_int32
    L.pinn_query.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_uint32, c_void_p,
                             c_void_p, c_size_t, c_void_p]
    L.pinn_exchange.restype = c_int32
    L.pinn_query_noalloc.restype = c_int32
    L.pinn_query_noalloc.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_uint32, c_void_p, c_void_p]
    L.pinn_exchange.argtypes = [c_void_p, POINTER(PinnFace), c_int32, POINTER(c_float),
                                POINTER(c_void_p), c_void_p]
    L.pinn_kernel_time.restype = c_int32
    L.pinn_kernel_time.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int64)]
    L.pinn_check_guards.restype = c_int32
    L.pinn_check_guards.argtypes = [c_void_p, POINTER(c_int64), c_void_p]
    L.pinn_evaluate_scratch_bytes.restype = c_size_t
    L.pinn_evaluate_scratch_bytes.argtypes = [c_void_p, c_int64, c_int32, c_int64]
    L.pinn_evaluate.restype = c_int32
    L.pinn_evaluate.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, POINTER(c_int64), c_int32,
                                POINTER(c_float), c_void_p, c_void_p, c_size_t, c_void_p]
    L.pinn_refresh.restype = c_int32
    L.pinn_refresh.argtypes = [c_void_p, c_void_p]
    L.pinn_destroy.restype = c_int32
    L.pinn_destroy.argtypes = [c_void_p]
    L.pinn_get_launch_info.restype = c_int32
    L.pinn_get_launch_info.argtypes = [c_void_p, POINTER(PinnLaunchInfo)]
    L.pinn_last_error.restype = c_char_p
    L.pinn_last_error.argtypes = []
    _lib = L
    return L


def check(status: int):
    if status != PINN_OK:
        raise PinnError(status, lib().pinn_last_error().decode())
    return status


def num_params(dim: int, width: int, depth: int) -> int:
    return int(lib().pinn_num_params(dim, width, depth))
