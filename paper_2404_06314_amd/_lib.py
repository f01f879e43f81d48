"""ctypes loader for libqtm.so: declares every C-ABI entry point of qtm.h.

There is no fallback: if the library is missing, importing the package's
compute entry points raises.
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libqtm.so"

QTM_OK = 0
QTM_ERR_INVALID_ARG = -1
QTM_ERR_UNSUPPORTED = -2
QTM_ERR_WORKSPACE = -3
QTM_ERR_HIP = -4
QTM_ERR_STATE = -5

QTM_RX, QTM_RY, QTM_RZ, QTM_CNOT, QTM_CZ = 0, 1, 2, 3, 4
QTM_H, QTM_X, QTM_Y, QTM_Z, QTM_S, QTM_SDG, QTM_T, QTM_TDG, QTM_SX = range(5, 14)
QTM_CRX, QTM_CRY, QTM_CRZ = 14, 15, 16
QTM_SRC_NONE, QTM_SRC_INPUT, QTM_SRC_WEIGHT, QTM_SRC_SCALED = 0, 1, 2, 3
QTM_C64, QTM_C128 = 0, 1
QTM_PATH_AUTO, QTM_PATH_PLAIN, QTM_PATH_FUSED = 0, 1, 2
QTM_OPT_PATH, QTM_OPT_TILE_QUBITS, QTM_OPT_LOW_QUBITS, QTM_OPT_RENORM, QTM_OPT_TIMING = 0, 1, 2, 3, 4
QTM_OPT_JIT = 5
QTM_OPT_CHECK_ANGLES = 6
QTM_OPT_DENSE_BLOCKS = 7
QTM_OPT_GREEDY_PLAN = 8
QTM_OPT_PLAN_IO = 9
QTM_OPT_JAC_CHUNK = 10

# every exported function of include/qtm.h: name -> (restype, argtypes)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
SIGNATURES = {
    "qtm_circuit_create": (ctypes.c_int, [_I32, _P, _I32, _I32, _I32, _P, _I32, _P]),
    "qtm_circuit_create_pauli": (ctypes.c_int, [_I32, _P, _I32, _I32, _I32, _P, _P, _I32, _P]),
    "qtm_circuit_destroy": (ctypes.c_int, [_P]),
    "qtm_set_option": (ctypes.c_int, [_P, _I32, _I64]),
    "qtm_state_bytes": (ctypes.c_int, [_P, _I32, _I32, _P]),
    "qtm_forward": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P, _P, _P]),
    "qtm_forward_noalloc": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P, _P, _P]),
    "qtm_backward": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "qtm_multi_create": (ctypes.c_int, [_P, _I32, _P]),
    "qtm_multi_destroy": (ctypes.c_int, [_P]),
    "qtm_multi_layout": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "qtm_multi_forward": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "qtm_multi_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "qtm_multi_set_option": (ctypes.c_int, [_P, _I32, ctypes.c_int64]),
    "qtm_multi_timing_read": (ctypes.c_int, [_P, _I32, _P, _P]),
    "qtm_multi_units": (ctypes.c_int, [_P, _I32, _P]),
    "qtm_timing_read": (ctypes.c_int, [_P, _I32, _P, _P]),
    "qtm_forward_norms": (ctypes.c_int, [_P, _I32, _P, _P]),
    "qtm_jit_source": (ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.c_char_p, _SZ, _P]),
    "qtm_jit_compile": (ctypes.c_int, [_P, _I32]),
    "qtm_jacobian": (ctypes.c_int, [_P, _I32, _I32, _P, _P, _P, _P, _P, _P]),
    "qtm_autotune": (ctypes.c_int, [_P, _I32, _I32, _P, _I32, ctypes.c_char_p, _SZ, _P]),
    "qtm_jit_info": (ctypes.c_int, [_P, _I32, _I32, _I32, _P, _P]),
    "qtm_plan_json": (ctypes.c_int, [_P, _I32, ctypes.c_char_p, _SZ, _P]),
    "qtm_last_error": (ctypes.c_char_p, []),
    "qtm_version": (ctypes.c_char_p, []),
}

_lib = None


class QtmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qtm error {code}: {msg}")
        self.code = code


def load():
    """Load libqtm.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2404_06314_amd.build` (no CPU fallback exists)")
        # One HIP runtime per process: torch's libraries name the runtime by
        # a different file name than libqtm does, so if libqtm were loaded
        # first the process would end up with two HIP/HSA runtimes and the
        # second one to initialise would see no device.  Loading torch first
        # makes libqtm bind to the runtime torch already holds.
        import torch  # noqa: F401
        lib = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(rc: int):
    if rc != QTM_OK:
        msg = load().qtm_last_error().decode(errors="replace")
        raise QtmError(rc, msg)
