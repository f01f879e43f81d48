"""Periodic FP64 renormalisation (QTM_OPT_RENORM = R): every R sweeps the
forward rescales the state to norm 1 by the previous sweep's FP64 norm, and
the backward rescales psi and lambda by the FP64 load / end norm ratios of
the sweeps since the last rescaling.  Every gate is linear, so the results
equal the unrenormalised ones up to rounding: against the oracle at the
same bar, on deep circuits, at 26 qubits, for the compiled and the
specialised kernels (including sweeps that skip unexcited qubits)."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_helpers import assert_parity, run_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


_REFS = {}


def _ref(wl, key):
    import oracle
    if key not in _REFS:
        _REFS[key] = oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)
    return _REFS[key]


def _circ(circ, jit, period, tile=None, klo=None):
    import paper_2404_06314_amd as q
    c = q.Circuit.from_workload(circ)
    c.set_option(q.QTM_OPT_JIT, jit)
    c.set_option(q.QTM_OPT_RENORM, period)
    if tile:
        c.set_option(q.QTM_OPT_TILE_QUBITS, tile)
    if klo:
        c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    return c


@pytest.mark.parametrize("precision,jit,period", [("c64", 0, 1), ("c64", 1, 1), ("c64", 1, 3),
                                                  ("c64", 0, 2), ("c128", 0, 1)])
def test_deep_circuit(precision, jit, period):
    """n = 14, 64 layers (3584 gates), tile 10: many sweeps per pass."""
    rng = np.random.default_rng(64)
    wl = W.random_workload(rng, W.layered_circuit(14, 64, "ring"), 4)
    c = _circ(wl.circuit, jit, period, 10, 4)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=c)
    assert_parity(got, _ref(wl, "deep"), precision, f"renorm n14 L64 {precision} jit={jit} R={period}")


@pytest.mark.parametrize("jit,period", [(1, 1), (0, 2)])
def test_c5_two_samples(jit, period):
    """n = 26, 10 layers, CNOT ring, complex64 against the oracle fixture."""
    d = np.load(os.path.join(GOLDEN, "oracle_c5_b2.npz"), allow_pickle=False)
    wl = W.config_workload("c5", batch=2)
    c = _circ(wl.circuit, jit, period)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64", qcirc=c)
    assert_parity(got, (d["expvals"], d["grad_w"], d["grad_x"]), "c64", f"renorm c5 jit={jit} R={period}")


@pytest.mark.parametrize("period", [1, 2])
def test_zero_skipping_sweeps_and_rounding_only(period):
    """CZ ladder, n = 16, tile 11 (specialised sweeps that run part of the
    tiles and load part of the amplitudes): the oracle bar, and the
    renormalised results equal the plain ones to rounding."""
    rng = np.random.default_rng(1600 + period)
    wl = W.random_workload(rng, W.layered_circuit(16, 6, "ladder", extra_masks=(0xFFFF,)), 3)
    plain = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64",
                    qcirc=_circ(wl.circuit, 1, 0, 11, 4))
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64",
                  qcirc=_circ(wl.circuit, 1, period, 11, 4))
    assert_parity(got, _ref(wl, f"n16 {period}"), "c64", f"renorm n16 ladder R={period}")
    assert np.max(np.abs(got[0] - plain[0])) <= 1e-6
    assert np.max(np.abs(got[1] - plain[1])) <= 1e-5 * np.max(np.abs(plain[1]))
