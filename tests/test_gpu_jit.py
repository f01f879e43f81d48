"""Sweep kernels specialised for the circuit at run time (QTM_OPT_JIT):
the same parity bar against the oracle as the compiled kernels, on the
benchmark sizes and on gate mixes that exercise every generated op form."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_helpers import assert_parity, run_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def jit_circuit(circ, tile=None, klo=None):
    import paper_2404_06314_amd as q
    c = q.Circuit.from_workload(circ)
    c.set_option(q.QTM_OPT_JIT, 1)
    if tile:
        c.set_option(q.QTM_OPT_TILE_QUBITS, tile)
    if klo:
        c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    return c


def oracle_ref(wl):
    import oracle
    return oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_c1_ring(precision):
    wl = W.config_workload("c1")
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=jit_circuit(wl.circuit))
    assert_parity(got, oracle_ref(wl), precision, f"jit c1 {precision}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,L,ent,tile,klo", [(8, 3, "ring", 5, 3), (10, 2, "ladder", 6, 4),
                                              (9, 4, "ring", 0, 0), (12, 2, "ladder", 8, 5)])
def test_multi_sweep_layered(precision, n, L, ent, tile, klo):
    rng = np.random.default_rng(n * 100 + L)
    circ = W.layered_circuit(n, L, ent, extra_masks=((1 << n) - 1,))
    wl = W.random_workload(rng, circ, 5)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision,
                  qcirc=jit_circuit(circ, tile or None, klo or None))
    assert_parity(got, oracle_ref(wl), precision, f"jit n={n} L={L} {ent} {precision}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_circuits(precision, seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(6, 10))
    circ = W.random_circuit(rng, n, int(rng.integers(40, 90)))
    wl = W.random_workload(rng, circ, 3)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=jit_circuit(circ, 5, 2))
    assert_parity(got, oracle_ref(wl), precision, f"jit random seed={seed} {precision}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_c3_full_batch(precision):
    """n=20, 8 layers, CZ ladder, batch 64 against the oracle fixture; two
    runs give the same bits; the specialised kernels spill at most a few
    registers (the backward kernels sit at the 256-register limit that two
    workgroups per compute unit allow)."""
    path = os.path.join(GOLDEN, "oracle_c3_b64.npz")
    d = np.load(path, allow_pickle=False)
    ref = (d["expvals"], d["grad_w"], d["grad_x"])
    wl = W.config_workload("c3")
    c = jit_circuit(wl.circuit)
    a = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=c)
    assert_parity(a, ref, precision, f"jit c3 {precision}")
    b = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=c)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    for direction in (0, 1):
        for s in range(len(c.plan(precision)["sweeps"])):
            vg, sc = c.jit_info(precision, direction, s)
            print(f"c3 {precision} dir {direction} sweep {s}: {vg} VGPRs, {sc} B scratch")
            assert sc <= 64
