"""ctypes declarations of the C ABI in include/superneuro_mi.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnmi.so")

SN_OK, SN_EINVAL, SN_ENOMEM, SN_EDEVICE, SN_ESTATE, SN_ERANGE, SN_EINEXACT = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SN_OK", -1: "SN_EINVAL", -2: "SN_ENOMEM", -3: "SN_EDEVICE", -4: "SN_ESTATE",
                -5: "SN_ERANGE", -6: "SN_EINEXACT"}
PATH_AUTO, PATH_SMALL, PATH_STEP, PATH_PERSIST, PATH_DENSE, PATH_PUSH, PATH_DENSE_STEP = 0, 1, 2, 3, 4, 5, 6
PATH_DENSE_ROWS = 10
PATH_NAMES = {0: "auto", 1: "small", 2: "step", 3: "persist", 4: "dense", 5: "push", 6: "dense_step",
              7: "batch", 8: "dense_persist", 9: "dense_persist_i8", 10: "dense_rows"}

# Every symbol the header declares.
EXPORTS = [
    "sn_create_network", "sn_load_weights_delays", "sn_load_dense_weights", "sn_load_dense_rows_i8",
    "sn_set_input_spikes",
    "sn_set_input_spikes_device", "sn_run", "sn_synchronize", "sn_read_raster", "sn_read_state",
    "sn_read_raster_device", "sn_read_state_device",
    "sn_reset_state", "sn_set_path", "sn_set_slices", "sn_autotune", "sn_get_progress", "sn_destroy_network",
    "sn_last_error", "sn_set_stdp", "sn_read_weights",
    "sn_batch_create", "sn_batch_run", "sn_batch_destroy", "sn_batch_autotune",
    "sn_bptt_workspace_bytes", "sn_bptt_forward", "sn_bptt_backward", "sn_bptt_forward_noalloc",
]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class SnAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class SnNetDesc(ctypes.Structure):
    _fields_ = [
        ("n_neurons", ctypes.c_int32), ("n_trials", ctypes.c_int32), ("max_delay", ctypes.c_int32),
        ("threshold", ctypes.c_void_p), ("leak", ctypes.c_void_p), ("reset", ctypes.c_void_p),
        ("refractory", ctypes.c_void_p), ("amplitude", ctypes.c_void_p),
        ("threshold_scalar", ctypes.c_float), ("leak_scalar", ctypes.c_float),
        ("reset_scalar", ctypes.c_float), ("amplitude_scalar", ctypes.c_float),
        ("refractory_scalar", ctypes.c_uint8),
    ]


class SnStdpDesc(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("ltp", ctypes.c_float * 16), ("ltd", ctypes.c_float * 16),
                ("w_min", ctypes.c_float), ("w_max", ctypes.c_float)]


class SnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load():
    """Load the HIP library; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the simulator has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "sn_create_network": [ctypes.POINTER(SnNetDesc), ctypes.POINTER(SnAllocator), P, ctypes.POINTER(P)],
        "sn_load_weights_delays": [P, I64, P, P, P, P],
        "sn_load_dense_weights": [P, P, I32],
        "sn_load_dense_rows_i8": [P, I32, I32, P, I32],
        "sn_set_input_spikes": [P, I32, I32, P],
        "sn_set_input_spikes_device": [P, I32, I32, P],
        "sn_run": [P, I32],
        "sn_synchronize": [P],
        "sn_read_raster": [P, I32, I32, P],
        "sn_read_state": [P, P, P],
        "sn_read_raster_device": [P, I32, I32, P],
        "sn_read_state_device": [P, P, P],
        "sn_reset_state": [P],
        "sn_set_path": [P, I32],
        "sn_set_slices": [P, I32],
        "sn_autotune": [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "sn_set_stdp": [P, ctypes.POINTER(SnStdpDesc)],
        "sn_read_weights": [P, P],
        "sn_get_progress": [P, ctypes.POINTER(I32), ctypes.POINTER(I32)],
        "sn_batch_create": [P, I32, ctypes.POINTER(P)],
        "sn_batch_run": [P, I32],
        "sn_batch_autotune": [P, I32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.sn_destroy_network.argtypes = [P]
    lib.sn_destroy_network.restype = None
    lib.sn_batch_destroy.argtypes = [P]
    lib.sn_batch_destroy.restype = None
    lib.sn_last_error.argtypes = []
    lib.sn_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != SN_OK:
        raise SnError(status, load().sn_last_error().decode(errors="replace"))
