"""CPU complex128 oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it, and
it shares no code with the GPU path (see ``qtm_oracle.c`` for what it
computes and which passages of the paper each part follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "qtm_oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc + OpenMP."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fcx-limited-range", "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("QTM_ORACLE_LIB")  # planted-mistake variants (tests only)
        if path is None:
            if not _LIB.exists():
                build(force=True)
            path = str(_LIB)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i = ctypes.c_int
        common = [i, P, i, i, i, P, P, i, i, P, P]
        lib.qtm_oracle_forward.argtypes = common + [P, i, i]
        lib.qtm_oracle_vjp.argtypes = common + [P, P, P, P, P, i, i]
        lib.qtm_oracle_jacobian.argtypes = common + [P, P, P, i, i]
        lib.qtm_oracle_state.argtypes = [i, P, i, i, i, P, P, P]
        lib.qtm_oracle_uncompute.argtypes = [i, P, i, i, i, P, P, P]
        lib.qtm_oracle_split.argtypes = [i, i, i, P]
        for f in (lib.qtm_oracle_forward, lib.qtm_oracle_vjp, lib.qtm_oracle_jacobian,
                  lib.qtm_oracle_state, lib.qtm_oracle_uncompute, lib.qtm_oracle_split):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _xmasks(circ):
    """X-parts of the observables' Pauli strings, or None (all Z strings)."""
    xm = getattr(circ, "xmasks", None)
    return None if xm is None else np.ascontiguousarray(xm, dtype=np.uint64)


def _prep(circ, x, w):
    gates = np.ascontiguousarray(circ.gates, dtype=np.int32)
    masks = np.ascontiguousarray(circ.masks, dtype=np.uint64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, max(circ.n_inputs, 1)) \
        if circ.n_inputs > 0 else np.zeros((np.asarray(x).shape[0], 1))
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.size == 0:
        w = np.zeros(1)
    return gates, masks, x, w


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def forward(circ, x, w, threads: int | None = None, par_mode: int = 0):
    """Expectation values (B, M)."""
    lib = _load()
    gates, masks, x, w = _prep(circ, x, w)
    xm = _xmasks(circ)
    B = x.shape[0]
    out = np.zeros((B, circ.n_obs))
    rc = lib.qtm_oracle_forward(circ.n, _ptr(gates), circ.n_gates, circ.n_inputs,
                                circ.n_weights, _ptr(masks), _ptr(xm), circ.n_obs, B,
                                _ptr(x), _ptr(w), _ptr(out),
                                threads or default_threads(), par_mode)
    if rc:
        raise RuntimeError(f"oracle forward failed ({rc})")
    return out


def vjp(circ, x, w, G, threads: int | None = None, par_mode: int = 0,
        occurrences: bool = False):
    """Returns (expvals (B,M), grad_w (n_w,), grad_x (B,n_in)[, g_occ (B,n_gates)])."""
    lib = _load()
    gates, masks, x, w = _prep(circ, x, w)
    xm = _xmasks(circ)
    B = x.shape[0]
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(B, circ.n_obs)
    out = np.zeros((B, circ.n_obs))
    gw = np.zeros(max(circ.n_weights, 1))
    gx = np.zeros((B, max(circ.n_inputs, 1)))
    gocc = np.zeros((B, max(circ.n_gates, 1))) if occurrences else None
    rc = lib.qtm_oracle_vjp(circ.n, _ptr(gates), circ.n_gates, circ.n_inputs,
                            circ.n_weights, _ptr(masks), _ptr(xm), circ.n_obs, B,
                            _ptr(x), _ptr(w), _ptr(G), _ptr(out), _ptr(gw), _ptr(gx),
                            _ptr(gocc), threads or default_threads(), par_mode)
    if rc:
        raise RuntimeError(f"oracle vjp failed ({rc})")
    res = (out, gw[:circ.n_weights], gx[:, :circ.n_inputs])
    if occurrences:
        res = res + (gocc[:, :circ.n_gates],)
    return res


def jacobian(circ, x, w, threads: int | None = None, par_mode: int = 0):
    """Returns (expvals (B,M), J_w (B,M,n_w), J_x (B,M,n_in))."""
    lib = _load()
    gates, masks, x, w = _prep(circ, x, w)
    xm = _xmasks(circ)
    B = x.shape[0]
    out = np.zeros((B, circ.n_obs))
    jw = np.zeros((B, circ.n_obs, max(circ.n_weights, 1)))
    jx = np.zeros((B, circ.n_obs, max(circ.n_inputs, 1)))
    rc = lib.qtm_oracle_jacobian(circ.n, _ptr(gates), circ.n_gates, circ.n_inputs,
                                 circ.n_weights, _ptr(masks), _ptr(xm), circ.n_obs, B,
                                 _ptr(x), _ptr(w), _ptr(out), _ptr(jw), _ptr(jx),
                                 threads or default_threads(), par_mode)
    if rc:
        raise RuntimeError(f"oracle jacobian failed ({rc})")
    return out, jw[:, :, :circ.n_weights], jx[:, :, :circ.n_inputs]


def state(circ, x_b, w):
    """Final state U|0> (complex128, length 2^n) of one sample."""
    lib = _load()
    gates, masks, x, w = _prep(circ, np.asarray(x_b).reshape(1, -1), w)
    buf = np.zeros(2 << circ.n)
    rc = lib.qtm_oracle_state(circ.n, _ptr(gates), circ.n_gates, circ.n_inputs,
                              circ.n_weights, _ptr(x), _ptr(w), _ptr(buf))
    if rc:
        raise RuntimeError(f"oracle state failed ({rc})")
    return buf[0::2] + 1j * buf[1::2]


def uncompute_residual(circ, x_b, w) -> float:
    lib = _load()
    gates, masks, x, w = _prep(circ, np.asarray(x_b).reshape(1, -1), w)
    a = ctypes.c_double(0.0)
    rc = lib.qtm_oracle_uncompute(circ.n, _ptr(gates), circ.n_gates, circ.n_inputs,
                                  circ.n_weights, _ptr(x), _ptr(w), ctypes.byref(a))
    if rc:
        raise RuntimeError(f"oracle uncompute failed ({rc})")
    return a.value


def split(B: int, T: int):
    """Sample ranges [(lo, hi)] of the T workers (Sec. II-B)."""
    lib = _load()
    out = []
    buf = np.zeros(2, dtype=np.int32)
    for t in range(T):
        if lib.qtm_oracle_split(B, T, t, _ptr(buf)):
            raise ValueError("bad split arguments")
        out.append((int(buf[0]), int(buf[1])))
    return out
