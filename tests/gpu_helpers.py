"""Helpers for GPU tests: run the HIP path through the C ABI and compare."""
from __future__ import annotations

import json
import os

import numpy as np

TOL_Z_C64 = 1e-5        # absolute, per expectation value
TOL_G_C64 = 1e-4        # norm-wise relative per gradient vector
TOL_Z_C128 = 1e-12
TOL_G_C128 = 1e-10
# Absolute bound for gradient vectors whose exact value is (near) zero, where a
# relative bound is meaningless: a few rounding units of the amplitude type.
# It applies only to vectors with max|ref| below FLOOR_G / TOL_G (1e-2 for
# complex64, 1e-3 for complex128); larger vectors take the relative bound alone.
FLOOR_G_C64 = 1e-6
FLOOR_G_C128 = 1e-13


def grad_bound(scale, tol, floor):
    """Allowed max|got - ref| for a gradient vector with max|ref| = scale."""
    return floor if floor > 0.0 and scale < floor / tol else tol * scale


def report(what, **errs):
    """Print the measured errors of a parity check (and append them as a JSON
    line to $QTM_PARITY_LOG when set)."""
    line = " ".join(f"{k}={v:.3e}" for k, v in errs.items())
    print(f"parity {what}: {line}")
    path = os.environ.get("QTM_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps({"what": what, **{k: float(v) for k, v in errs.items()}}) + "\n")


def run_gpu(circ, x, w, G, precision="c64", path=None, tile=None, klo=None, keep_state=True,
            qcirc=None):
    """Forward + backward on cuda:0.  Returns numpy (expvals, grad_w, grad_x)."""
    import torch
    import paper_2404_06314_amd as q
    c = qcirc or q.Circuit.from_workload(circ)
    if path is not None:
        c.set_path(path)
    if tile:
        c.set_option(q.QTM_OPT_TILE_QUBITS, tile)
    if klo:
        c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    dev = torch.device("cuda:0")
    xt = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    wt = torch.as_tensor(np.ascontiguousarray(w), dtype=torch.float64, device=dev)
    Gt = torch.as_tensor(np.ascontiguousarray(G), dtype=torch.float64, device=dev)
    B = xt.shape[0]
    st = c.alloc_state(B, precision) if keep_state else None
    ev = c.forward(xt, wt, precision, state=st)
    gw, gx = c.backward(xt, wt, Gt, precision, state=st)
    torch.cuda.synchronize()
    return ev.cpu().numpy(), gw.cpu().numpy(), gx.cpu().numpy()


def assert_grad_close(got, ref, tol, what="", floor=0.0):
    """Norm-wise relative check per vector: max|got - ref| <= tol * max|ref|,
    or <= floor for vectors whose max|ref| is below floor / tol.  Returns the
    error relative to max|ref| (0 for an all-zero reference)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    err = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    bound = grad_bound(scale, tol, floor)
    assert err <= bound, f"{what}: max err {err:.3e} > {bound:.3e} (max|ref| {scale:.3e})"
    return err / scale if scale > 0.0 else 0.0


def assert_parity(gpu, ref, precision, what=""):
    ev, gw, gx = gpu
    rev, rgw, rgx = ref
    tz = TOL_Z_C64 if precision == "c64" else TOL_Z_C128
    tg = TOL_G_C64 if precision == "c64" else TOL_G_C128
    fl = FLOOR_G_C64 if precision == "c64" else FLOOR_G_C128
    err = np.max(np.abs(ev - rev))
    assert err <= tz, f"{what}: <Z> max err {err:.3e} > {tz:g}"
    rw = assert_grad_close(gw, rgw, tg, what + " dL/dw", fl) if rgw.size else 0.0
    rx = 0.0
    for b in range(rgx.shape[0]):
        if rgx.shape[1]:
            rx = max(rx, assert_grad_close(gx[b], rgx[b], tg, what + f" dL/dx[{b}]", fl))
    report(what, z_abs=err, gw_rel=rw, gx_rel=rx)
