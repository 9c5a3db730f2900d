"""ctypes binding of libdclbm.so (the C ABI in include/dclbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdclbm.so")

MAX_LEVELS = 4
ABI_VERSION = 5

LATTICE = {"D2Q9": 0, "D3Q19": 1}
PRECISION = {"fp64": 0, "fp32": 1, "fp16": 2}
COLLISION = {"bgk": 0, "hrr": 1}

STATUS = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "HIP", -4: "NEWTON", -5: "UNSTABLE", -6: "BUSY"}


class DclbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"dclbm {STATUS.get(status, status)}: {message}")
        self.status = status


class Config(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32),
        ("lattice", C.c_int32),
        ("precision", C.c_int32),
        ("coupling", C.c_int32),
        ("eq_order", C.c_int32),
        ("n0", C.c_int32 * 3),
        ("n_levels", C.c_int32),
        ("box_lo", (C.c_int32 * 3) * (MAX_LEVELS - 1)),
        ("box_hi", (C.c_int32 * 3) * (MAX_LEVELS - 1)),
        ("tau0", C.c_double),
        ("n_probes", C.c_int32),
        ("h_probe_xyz", C.POINTER(C.c_int32)),
        ("probe_capacity", C.c_int64),
        ("newton_max_iter", C.c_int32),
        ("newton_tol", C.c_double),
        ("u_ref", C.c_double * 3),
        ("collision", C.c_int32),
        ("hrr_sigma", C.c_double),
        ("hrr_psi", C.c_int32),
        ("sponge_cells", C.c_int32),
        ("sponge_sigma", C.c_double),
        ("h_region", C.POINTER(C.c_uint8)),
    ]


class ServerConfig(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32),
        ("lattice", C.c_int32),
        ("precision", C.c_int32),
        ("eq_order", C.c_int32),
        ("max_levels", C.c_int32),
        ("max_slots", C.c_int32),
        ("steps_per_tick", C.c_int32),
        ("max_probes", C.c_int32),
        ("max_probe_steps", C.c_int64),
        ("max_level_nodes", C.c_int64),
        ("grid", C.c_int32),
        ("max_inflight", C.c_int32),
    ]


class RequestInfo(C.Structure):
    _fields_ = [
        ("t_submit", C.c_double),
        ("t_admit", C.c_double),
        ("t_done", C.c_double),
        ("steps", C.c_int64),
        ("updates", C.c_int64),
        ("workspace_bytes", C.c_int64),
        ("slot", C.c_int32),
        ("state", C.c_int32),
        ("status", C.c_int32),
        ("n_probes", C.c_int32),
    ]


class ServerInfo(C.Structure):
    _fields_ = [
        ("ticks", C.c_int64),
        ("running", C.c_int32),
        ("queued", C.c_int32),
        ("arena_bytes", C.c_int64),
        ("arena_free", C.c_int64),
        ("arena_largest_free", C.c_int64),
        ("grid", C.c_int32),
        ("n_phases", C.c_int32),
    ]


REQ_STATE = {0: "queued", 1: "running", 2: "done", 3: "failed"}

_lock = threading.Lock()
_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "dclbm_workspace_bytes": (C.c_int, [C.POINTER(Config), C.POINTER(C.c_size_t)]),
    "dclbm_create": (C.c_int, [C.POINTER(Config), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "dclbm_destroy": (C.c_int, [C.c_void_p]),
    "dclbm_level_shape": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "dclbm_updates_per_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "dclbm_init_equilibrium": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dclbm_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "dclbm_check": (C.c_int, [C.c_void_p]),
    "dclbm_read_populations": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "dclbm_read_macros": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dclbm_read_shared": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "dclbm_velocity_divergence": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dclbm_read_probes": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]),
    "dclbm_set_probe_window": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64]),
    "dclbm_read_probe_sums": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]),
    "dclbm_balance": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "dclbm_balance_static": (C.c_int, [C.c_void_p, C.c_void_p]),
    "dclbm_interface_bytes": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "dclbm_checkpoint_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "dclbm_save": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "dclbm_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "dclbm_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "dclbm_set_split": (C.c_int, [C.c_void_p, C.c_int32]),
    "dclbm_bulk_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)]),
    "dclbm_copy_calibration": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_int32,
                                         C.POINTER(C.c_double)]),
    "dclbm_lattice_table": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double)]),
    "dclbm_last_error": (C.c_char_p, []),
    "dclbm_server_workspace_bytes": (C.c_int, [C.POINTER(ServerConfig), C.c_size_t, C.POINTER(C.c_size_t)]),
    "dclbm_server_create": (C.c_int, [C.POINTER(ServerConfig), C.c_void_p, C.c_size_t, C.c_void_p,
                                      C.POINTER(C.c_void_p)]),
    "dclbm_server_destroy": (C.c_int, [C.c_void_p]),
    "dclbm_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Config), C.c_int64, C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_void_p), C.POINTER(C.c_uint64)]),
    "dclbm_server_tick": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "dclbm_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]),
    "dclbm_server_result": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.POINTER(C.c_int64),
                                      C.POINTER(RequestInfo)]),
    "dclbm_server_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "dclbm_server_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerInfo)]),
}


def load():
    """Load the built library; raises if it is missing (build it with
    __graft_entry__.build() or paper_2004_14887_amd/build.py)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"HIP library not built: {LIB_PATH} is missing")
            lib = C.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(status: int):
    if status != 0:
        msg = load().dclbm_last_error()
        raise DclbmError(status, msg.decode() if msg else "")


def exported_symbols():
    lib = load()
    return {name for name in _SIGS if hasattr(lib, name)}
