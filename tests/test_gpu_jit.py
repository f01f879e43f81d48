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
@pytest.mark.parametrize("n,L,ent,B", [(5, 3, "ring", 7), (6, 2, "ladder", 3), (12, 2, "ring", 5)])
def test_single_tile_samples_write_expectations_directly(precision, n, L, ent, B):
    # tile = n: one workgroup holds a whole sample, and the last forward sweep
    # divides by the norm itself instead of leaving partial rows (at n = 5 a
    # workgroup has 2 threads for 9 observables, so each thread takes several)
    rng = np.random.default_rng(40 + n)
    masks = ((1 << n) - 1, 0b101, 0b11 << (n - 2), 1 << (n - 1))
    circ = W.layered_circuit(n, L, ent, extra_masks=masks)
    wl = W.random_workload(rng, circ, B)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=jit_circuit(circ, n))
    assert_parity(got, oracle_ref(wl), precision, f"jit single tile n={n} B={B} {precision}")


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
    registers (the backward kernels are built for three workgroups per
    compute unit, 168 registers, and rebuilt with two LDS tiles if they
    would spill)."""
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


@pytest.mark.parametrize("tile,klo", [(10, 4), (11, 3), (11, 4), (12, 5)])
def test_matrix_core_ladder_tiles(tile, klo):
    """CZ-ladder circuits through the matrix-core specialised sweeps (tiles of
    10-12 qubits) at several low-qubit counts."""
    rng = np.random.default_rng(tile * 10 + klo)
    circ = W.layered_circuit(14, 4, "ladder", extra_masks=(0b11 << 6, (1 << 14) - 1))
    wl = W.random_workload(rng, circ, 4)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, "c64", qcirc=jit_circuit(circ, tile, klo))
    assert_parity(got, oracle_ref(wl), "c64", f"jit ladder t{tile}l{klo}")


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_matrix_core_random_cz_heavy(seed):
    """Random circuits where half the gates are CZ (between any qubits), the
    rest rotations and CNOTs, through the matrix-core specialised sweeps."""
    rng = np.random.default_rng(900 + seed)
    n = 12
    g = []
    for _ in range(160):
        r = rng.random()
        if r < 0.5:
            a, b = rng.choice(n, size=2, replace=False)
            g.append((W.CZ, int(a), int(b), 0, 0))
        elif r < 0.6:
            a, b = rng.choice(n, size=2, replace=False)
            g.append((W.CNOT, int(a), int(b), 0, 0))
        else:
            t = int(rng.integers(0, 3))
            src = W.SRC_INPUT if rng.random() < 0.3 else W.SRC_WEIGHT
            g.append((t, int(rng.integers(0, n)), 0, src, int(rng.integers(0, 4))))
    circ = W.Circuit(n=n, gates=np.array(g, np.int32), n_inputs=4, n_weights=4,
                     masks=rng.integers(1, 1 << n, size=5, dtype=np.uint64))
    wl = W.random_workload(rng, circ, 3)
    t, k = [(10, 2), (11, 4), (12, 3), (10, 5)][seed - 1]
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, "c64", qcirc=jit_circuit(circ, t, k))
    assert_parity(got, oracle_ref(wl), "c64", f"jit cz-heavy seed={seed} t{t}l{k}")


def test_c3_runner_up_configuration():
    """The n=20 workload at tile 11 / 4 low qubits (specialised sweeps), one
    of the autotuner's candidates, against the oracle fixture.  The
    configuration the benchmark times after tuning (tile 12 / 4 low qubits,
    zero-skip plan) runs in test_c3_sweep_plans; the library's default tile
    (12 / 5 low qubits) in test_c3_full_batch."""
    d = np.load(os.path.join(GOLDEN, "oracle_c3_b64.npz"), allow_pickle=False)
    wl = W.config_workload("c3")
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64",
                  qcirc=jit_circuit(wl.circuit, 11, 4))
    assert_parity(got, (d["expvals"], d["grad_w"], d["grad_x"]), "c64", "jit c3 t11l4")


@pytest.mark.parametrize("jit", [0, 1])
@pytest.mark.parametrize("n,L,ent,klo", [(12, 3, "ring", 5), (14, 2, "ladder", 4)])
def test_c128_tile12(jit, n, L, ent, klo):
    """complex128 with 12-qubit tiles (the option and the autotuner accept
    them; the default complex128 tile is 11): generic and specialised sweeps,
    one tile per sample (n = 12) and several (n = 14)."""
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(1200 + n)
    circ = W.layered_circuit(n, L, ent, extra_masks=((1 << n) - 1,))
    wl = W.random_workload(rng, circ, 3)
    c = q.Circuit.from_workload(circ)
    c.set_option(q.QTM_OPT_JIT, jit)
    c.set_option(q.QTM_OPT_TILE_QUBITS, 12)
    c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, "c128", qcirc=c)
    assert c.plan("c128")["kt"] == 12
    assert_parity(got, oracle_ref(wl), "c128", f"c128 tile 12 n={n} jit={jit}")


@pytest.mark.parametrize("klo,greedy", [(4, 0), (3, 0), (5, 1)])
def test_c3_sweep_plans(klo, greedy):
    """The n=20 workload through the specialised sweeps with the plan chosen
    for skipping all-zero tiles (the default with QTM_OPT_JIT; 3 and 4 low
    qubits) and with the greedy plan (QTM_OPT_GREEDY_PLAN), against the oracle
    fixture."""
    import paper_2404_06314_amd as q
    d = np.load(os.path.join(GOLDEN, "oracle_c3_b64.npz"), allow_pickle=False)
    wl = W.config_workload("c3")
    c = jit_circuit(wl.circuit, 12, klo)
    c.set_option(q.QTM_OPT_GREEDY_PLAN, greedy)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64", qcirc=c)
    assert_parity(got, (d["expvals"], d["grad_w"], d["grad_x"]), "c64", f"jit c3 t12l{klo} greedy={greedy}")
