"""MI355X-native batched statevector forward + adjoint VJP (libqtm binding).

Thin Python layer over the C ABI in ``include/qtm.h``: it marshals torch
device tensors into plain pointers and the current HIP stream; every step of
the computation runs in the HIP kernels of ``libqtm.so``.
"""
from __future__ import annotations

import ctypes
import json

import numpy as np

from . import _lib
from ._lib import (QTM_C64, QTM_C128, QTM_CNOT, QTM_CZ, QTM_PATH_AUTO, QTM_PATH_FUSED,
                   QTM_PATH_PLAIN, QTM_RX, QTM_RY, QTM_RZ, QTM_SRC_INPUT, QTM_SRC_NONE,
                   QTM_SRC_SCALED, QTM_SRC_WEIGHT, QTM_OPT_LOW_QUBITS, QTM_OPT_PATH, QTM_OPT_RENORM,
                   QTM_OPT_TILE_QUBITS, QTM_OPT_TIMING, QTM_OPT_JIT, QTM_OPT_CHECK_ANGLES, QTM_OPT_DENSE_BLOCKS,
                   QTM_OPT_GREEDY_PLAN, QTM_OPT_PLAN_IO, QTM_OPT_JAC_CHUNK, QtmError)

__all__ = ["Circuit", "Multi", "QtmError", "precision_code", "lib_path",
           "QTM_C64", "QTM_C128", "QTM_PATH_AUTO", "QTM_PATH_PLAIN", "QTM_PATH_FUSED"]


def lib_path() -> str:
    return str(_lib.LIB_PATH)


def precision_code(p) -> int:
    if p in (QTM_C64, "c64", "complex64"):
        return QTM_C64
    if p in (QTM_C128, "c128", "complex128"):
        return QTM_C128
    raise ValueError(f"unknown precision {p!r}")


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Circuit:
    """A validated circuit handle (gate list + Pauli-string observables).

    ``masks`` are the observables' Z-parts; ``xmasks`` (optional) their
    X-parts: on qubit q the factor is X for bits (1, 0), Y for (1, 1), Z for
    (0, 1).  Without ``xmasks`` every observable is a Z string."""

    def __init__(self, n_qubits: int, gates, n_inputs: int, n_weights: int, masks, xmasks=None):
        lib = _lib.load()
        g = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 5))
        m = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64).reshape(-1))
        h = ctypes.c_void_p()
        if xmasks is None:
            _lib.check(lib.qtm_circuit_create(n_qubits, g.ctypes.data_as(ctypes.c_void_p), g.shape[0],
                                              n_inputs, n_weights, m.ctypes.data_as(ctypes.c_void_p),
                                              m.shape[0], ctypes.byref(h)))
            xm = None
        else:
            xm = np.ascontiguousarray(np.asarray(xmasks, dtype=np.uint64).reshape(-1))
            if xm.shape != m.shape:
                raise ValueError("xmasks and masks must have the same length")
            _lib.check(lib.qtm_circuit_create_pauli(
                n_qubits, g.ctypes.data_as(ctypes.c_void_p), g.shape[0], n_inputs, n_weights,
                xm.ctypes.data_as(ctypes.c_void_p), m.ctypes.data_as(ctypes.c_void_p), m.shape[0],
                ctypes.byref(h)))
        self.xmasks = xm
        self._h = h
        self.n = int(n_qubits)
        self.gates = g
        self.masks = m
        self.n_inputs = int(n_inputs)
        self.n_weights = int(n_weights)
        self.n_obs = int(m.shape[0])

    @classmethod
    def from_workload(cls, circ):
        """From a ``workloads.Circuit``-like object (n, gates, n_inputs, n_weights, masks
        and optionally xmasks)."""
        return cls(circ.n, circ.gates, circ.n_inputs, circ.n_weights, circ.masks,
                   getattr(circ, "xmasks", None))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().qtm_circuit_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: int):
        _lib.check(_lib.load().qtm_set_option(self._h, option, int(value)))

    def set_path(self, path: int):
        self.set_option(QTM_OPT_PATH, path)

    def state_bytes(self, batch: int, precision=QTM_C64) -> int:
        out = ctypes.c_size_t()
        _lib.check(_lib.load().qtm_state_bytes(self._h, batch, precision_code(precision),
                                               ctypes.byref(out)))
        return int(out.value)

    def plan(self, precision=QTM_C64) -> dict:
        """The fused-path plan (qtm_plan_json): sweeps with their tile qubits
        and stages, the encoded program (code, thr, sweep offsets) and, per
        sweep, the mask of qubits excited by its end (excited)."""
        lib = _lib.load()
        need = ctypes.c_size_t()
        _lib.check(lib.qtm_plan_json(self._h, precision_code(precision), None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _lib.check(lib.qtm_plan_json(self._h, precision_code(precision), buf, need.value,
                                     ctypes.byref(need)))
        return json.loads(buf.value.decode())

    def jit_source(self, precision=QTM_C64, direction: int = 0, sweep: int = 0) -> str:
        """HIP source of the specialised kernel of one sweep (diagnostics)."""
        lib = _lib.load()
        need = ctypes.c_size_t()
        p = precision_code(precision)
        _lib.check(lib.qtm_jit_source(self._h, p, direction, sweep, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _lib.check(lib.qtm_jit_source(self._h, p, direction, sweep, buf, need.value, ctypes.byref(need)))
        return buf.value.decode()

    def jit_compile(self, precision=QTM_C64):
        """Compile the specialised sweep kernels now (no device needed)."""
        _lib.check(_lib.load().qtm_jit_compile(self._h, precision_code(precision)))

    def autotune(self, batch: int, precision=QTM_C64, cache: bool = True, stream=None) -> dict:
        """Search tile size, contiguous low qubits, generic / specialised
        sweep kernels and the sweep plan of the specialised ones (zero-skip
        or greedy) for (batch, precision); installs the fastest candidate
        that reproduces the complex128 per-gate result.  Returns the JSON
        report (candidates with timings and errors)."""
        lib = _lib.load()
        need = ctypes.c_size_t()
        buf = ctypes.create_string_buffer(1 << 16)
        rc = lib.qtm_autotune(self._h, int(batch), precision_code(precision), _stream_ptr(stream),
                              1 if cache else 0, buf, len(buf), ctypes.byref(need))
        _lib.check(rc)
        return json.loads(buf.value.decode())

    def jit_info(self, precision=QTM_C64, direction: int = 0, sweep: int = 0):
        """(vector registers, scratch bytes) of a loaded specialised kernel."""
        v = ctypes.c_int32()
        sc = ctypes.c_int32()
        _lib.check(_lib.load().qtm_jit_info(self._h, precision_code(precision), direction, sweep,
                                            ctypes.byref(v), ctypes.byref(sc)))
        return int(v.value), int(sc.value)

    # --- raw pointer calls ----------------------------------------------------
    def forward_ptr(self, batch, precision, inputs, weights, expvals, state, stream):
        _lib.check(_lib.load().qtm_forward(self._h, batch, precision, inputs, weights, expvals,
                                           state, stream))

    def backward_ptr(self, batch, precision, inputs, weights, grad_expvals, state, grad_weights,
                     grad_inputs, stream):
        _lib.check(_lib.load().qtm_backward(self._h, batch, precision, inputs, weights,
                                            grad_expvals, state, grad_weights, grad_inputs, stream))

    # --- torch tensors ----------------------------------------------------------
    def alloc_state(self, batch: int, precision=QTM_C64, device=None):
        import torch
        nbytes = self.state_bytes(batch, precision)
        return torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")

    def forward(self, inputs, weights, precision=QTM_C64, state=None, stream=None):
        """inputs (B, n_inputs) float64 cuda, weights (n_weights,) float64 cuda ->
        expvals (B, M) float64.  `state` (from alloc_state) keeps the final
        states for backward."""
        import torch
        B = int(inputs.shape[0])
        _check_f64(inputs, weights)
        out = torch.empty((B, self.n_obs), dtype=torch.float64, device=inputs.device)
        self.forward_ptr(B, precision_code(precision), _ptr(inputs), _ptr(weights), _ptr(out),
                         _ptr(state), _stream_ptr(stream))
        return out

    def backward(self, inputs, weights, grad_expvals, precision=QTM_C64, state=None,
                 need_inputs=True, stream=None):
        """Returns (grad_weights (n_weights,), grad_inputs (B, n_inputs) or None)."""
        import torch
        B = int(inputs.shape[0])
        _check_f64(inputs, weights, grad_expvals)
        gw = torch.empty((max(self.n_weights, 0),), dtype=torch.float64, device=inputs.device)
        gx = torch.empty((B, self.n_inputs), dtype=torch.float64, device=inputs.device) \
            if need_inputs else None
        self.backward_ptr(B, precision_code(precision), _ptr(inputs), _ptr(weights),
                          _ptr(grad_expvals), _ptr(state), _ptr(gw), _ptr(gx),
                          _stream_ptr(stream))
        return gw, gx

    def forward_norms(self, batch: int, stream=None):
        """Squared norms (B,) float64 of the final states of the last forward
        pass (qtm_forward_norms): 1 in exact arithmetic; the distance from 1
        is the rounding drift of the evolution."""
        import torch
        out = torch.empty((int(batch),), dtype=torch.float64, device="cuda")
        _lib.check(_lib.load().qtm_forward_norms(self._h, int(batch), _ptr(out), _stream_ptr(stream)))
        return out


def _jacobian(self, inputs, weights, precision=QTM_C64, need_inputs=True, stream=None):
    """Full Jacobian: (expvals (B, M), J_w (B, M, n_weights), J_x (B, M, n_inputs) or None)."""
    import torch
    B = int(inputs.shape[0])
    _check_f64(inputs, weights)
    dev = inputs.device
    out = torch.empty((B, self.n_obs), dtype=torch.float64, device=dev)
    jw = torch.empty((B, self.n_obs, max(self.n_weights, 0)), dtype=torch.float64, device=dev)
    jx = torch.empty((B, self.n_obs, self.n_inputs), dtype=torch.float64, device=dev) \
        if need_inputs else None
    _lib.check(_lib.load().qtm_jacobian(self._h, B, precision_code(precision), _ptr(inputs), _ptr(weights),
                                        _ptr(out), _ptr(jw), _ptr(jx), _stream_ptr(stream)))
    return out, jw, jx


Circuit.jacobian = _jacobian


def _check_f64(*ts):
    import torch
    for t in ts:
        if t is None:
            continue
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise TypeError("expected contiguous float64 cuda tensors")


class Multi:
    """Uneven batch: one sample per circuit, circuits of any size and depth.

    Items of 4 or more qubits run in one persistent kernel per direction,
    launched as a HIP graph; item i owns the slices [in_off[i], in_off[i+1])
    of the packed inputs and input gradients, [w_off[i], w_off[i+1]) of the
    packed weights and weight gradients, and [out_off[i], out_off[i+1]) of the
    packed expectation values and their upstream gradients.
    """

    def __init__(self, circuits):
        lib = _lib.load()
        self.items = list(circuits)
        arr = (ctypes.c_void_p * max(len(self.items), 1))(*[c.handle.value for c in self.items])
        h = ctypes.c_void_p()
        _lib.check(lib.qtm_multi_create(arr, len(self.items), ctypes.byref(h)))
        self._h = h
        k = len(self.items) + 1
        self.in_off = np.zeros(k, np.int64)
        self.w_off = np.zeros(k, np.int64)
        self.out_off = np.zeros(k, np.int64)
        sb = ctypes.c_size_t()
        _lib.check(lib.qtm_multi_layout(h, self.in_off.ctypes.data_as(ctypes.c_void_p),
                                        self.w_off.ctypes.data_as(ctypes.c_void_p),
                                        self.out_off.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(sb)))
        self.state_bytes = int(sb.value)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().qtm_multi_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, on: bool):
        _lib.check(_lib.load().qtm_multi_set_option(self._h, QTM_OPT_TIMING, 1 if on else 0))

    def timing_read(self, kind: int):
        """(total ms, launches) of the persistent kernel of pass `kind` since the last read."""
        ms = ctypes.c_double()
        nl = ctypes.c_int64()
        _lib.check(_lib.load().qtm_multi_timing_read(self._h, kind, ctypes.byref(ms),
                                                     ctypes.byref(nl)))
        return ms.value, nl.value

    def units(self, kind: int) -> int:
        u = ctypes.c_int64()
        _lib.check(_lib.load().qtm_multi_units(self._h, kind, ctypes.byref(u)))
        return int(u.value)

    def alloc_state(self, device=None):
        import torch
        return torch.empty(max(self.state_bytes, 1), dtype=torch.uint8, device=device or "cuda")

    def forward(self, inputs, weights, state, stream=None):
        """Packed inputs / weights (float64 cuda) -> packed expvals (float64)."""
        import torch
        _check_f64(inputs, weights)
        out = torch.empty(int(self.out_off[-1]), dtype=torch.float64, device=state.device)
        _lib.check(_lib.load().qtm_multi_forward(self._h, _ptr(inputs), _ptr(weights), _ptr(out),
                                                 _ptr(state), _stream_ptr(stream)))
        return out

    def backward(self, inputs, weights, grad_expvals, state, need_inputs=True, stream=None):
        """Returns packed (grad_weights, grad_inputs or None); consumes `state`."""
        import torch
        _check_f64(inputs, weights, grad_expvals)
        dev = state.device
        gw = torch.empty(int(self.w_off[-1]), dtype=torch.float64, device=dev)
        gx = torch.empty(int(self.in_off[-1]), dtype=torch.float64, device=dev) \
            if need_inputs else None
        _lib.check(_lib.load().qtm_multi_backward(self._h, _ptr(inputs), _ptr(weights),
                                                  _ptr(grad_expvals), _ptr(state), _ptr(gw),
                                                  _ptr(gx), _stream_ptr(stream)))
        return gw, gx
