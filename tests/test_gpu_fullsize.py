"""GPU parity at the full benchmark sizes, in the launch configuration bench.py
times, against oracle results written by tests/golden/make_oracle_fixtures.py
(which calls only the oracle), plus the parameter-shift check of the n = 12
configuration and properties that hold at any size."""
import os

import numpy as np
import pytest

import workloads as W
import checkers as C
from gpu_helpers import assert_grad_close, assert_parity, run_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def fixture(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} missing: run tests/golden/make_oracle_fixtures.py")
    d = np.load(path, allow_pickle=False)
    return d["expvals"], d["grad_w"], d["grad_x"]


@pytest.mark.parametrize("precision,path", [("c64", None), ("c128", None), ("c128", 1)])
def test_c3_full_batch(precision, path):
    """n=20, 8 layers, CZ ladder, batch 64: every output against the oracle."""
    wl = W.config_workload("c3")
    ref = fixture("oracle_c3_b64.npz")
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, path)
    assert_parity(got, ref, precision, f"c3 {precision} path={path}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_c5_two_samples(precision):
    """n=26, 10 layers, CNOT ring: a 2-sample batch against the oracle."""
    wl = W.config_workload("c5", batch=2)
    ref = fixture("oracle_c5_b2.npz")
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision)
    assert_parity(got, ref, precision, f"c5 {precision}")


def test_c5_full_batch_sampled_and_linear():
    """n=26, batch 16 (complex64): the first two samples' outputs match the
    oracle, and dL/dw of the batch equals the sum over two sub-batches."""
    wl = W.config_workload("c5")
    rev, rgw2, rgx = fixture("oracle_c5_b2.npz")
    ev, gw, gx = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64")
    assert np.max(np.abs(ev[:2] - rev)) <= 1e-5
    for b in range(2):
        assert_grad_close(gx[b], rgx[b], 1e-4, f"c5 dL/dx[{b}]", 1e-6)
    _, gwa, _ = run_gpu(wl.circuit, wl.inputs[:2], wl.weights, wl.grad_out[:2], "c64")
    _, gwb, _ = run_gpu(wl.circuit, wl.inputs[2:], wl.weights, wl.grad_out[2:], "c64")
    assert_grad_close(gwa, rgw2, 1e-4, "c5 dL/dw first two", 1e-6)
    assert_grad_close(gw, gwa + gwb, 1e-5, "c5 dL/dw linearity", 1e-7)


def test_c2_adjoint_vs_parameter_shift():
    """n=12, 4 layers, ring: the autograd Function's gradient equals the
    parameter-shift gradient, both on the GPU.  Every rotation occurrence gets
    its own input slot; one batched forward evaluates all +-pi/2 shifts."""
    import torch
    import paper_2404_06314_amd as q
    from paper_2404_06314_amd.autograd import QtmFunction
    wl = W.config_workload("c2", batch=4)
    c = q.Circuit.from_workload(wl.circuit)
    x = torch.tensor(wl.inputs, device="cuda", requires_grad=True)
    w = torch.tensor(wl.weights, device="cuda", requires_grad=True)
    G = torch.tensor(wl.grad_out, device="cuda")
    out = QtmFunction.apply(x, w, c, "c64")
    (out * G).sum().backward()
    gw_adj = w.grad.cpu().numpy()
    gx_adj = x.grad.cpu().numpy()
    gw_ps = np.zeros_like(gw_adj)
    gx_ps = np.zeros_like(gx_adj)
    for b in range(wl.batch):
        cu, base, occ = C.untie_to_inputs(wl.circuit, wl.inputs[b], wl.weights)
        qc = q.Circuit.from_workload(cu)
        K = len(occ)
        rows = np.repeat(base[None, :], 2 * K, axis=0)
        rows[np.arange(K), np.arange(K)] += np.pi / 2
        rows[K + np.arange(K), np.arange(K)] -= np.pi / 2
        ev = qc.forward(torch.tensor(rows, device="cuda"),
                        torch.zeros(1, dtype=torch.float64, device="cuda"), "c64").cpu().numpy()
        d = (ev[:K] - ev[K:]) / 2 @ wl.grad_out[b]          # per occurrence
        for k, gi in enumerate(occ):
            t, q0, q1, src, idx = wl.circuit.gates[gi]
            if src == W.SRC_WEIGHT:
                gw_ps[idx] += d[k]
            else:
                gx_ps[b, idx] += d[k]
    assert_grad_close(gw_adj, gw_ps, 1e-4, "c2 dL/dw adjoint vs shift", 1e-6)
    for b in range(wl.batch):
        assert_grad_close(gx_adj[b], gx_ps[b], 1e-4, f"c2 dL/dx[{b}] adjoint vs shift", 1e-6)


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_c3_repeats_are_bitwise_identical(precision):
    """Four forward + backward runs of the full n=20 batch give the same bits
    (every reduction has a fixed order), and match the oracle.  Guards the
    backward sweep's LDS accumulators, which must be cleared before any wave
    adds its first-sweep norm partial."""
    wl = W.config_workload("c3")
    ref = fixture("oracle_c3_b64.npz")
    first = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision)
    assert_parity(first, ref, precision, f"c3 {precision} run 0")
    for rep in range(1, 4):
        got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision)
        for a, b in zip(first, got):
            assert np.array_equal(a, b), f"c3 {precision}: run {rep} differs from run 0"


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_max_qubits_n30_closed_form(precision):
    """The largest circuit the library accepts (30 qubits, 8 GiB of complex64
    amplitudes per sample): one RX / RY / RZ layer, a CZ ladder, then a CNOT
    ring.  The CZs commute with every Z string and the CNOT ring maps a Z
    string S to the Z string S' (Heisenberg picture), so <Z_S> is the product
    of the z parts of the single-qubit Bloch vectors over S', and so is its
    gradient (Bloch closed form), independent of the oracle."""
    n, B = 30, 2
    rng = np.random.default_rng(30)
    single = W.layered_circuit(n, 1, "none")
    ladder = [[W.CZ, i, i + 1, 0, 0] for i in range(n - 1)]
    ring = [(i, (i + 1) % n) for i in range(n)]
    gates = np.concatenate([single.gates, np.array(ladder, np.int32),
                            np.array([[W.CNOT, c, t, 0, 0] for c, t in ring], np.int32)])
    masks = [1 << q for q in range(0, n, 3)] + [(1 << 29) | 1, 0b1011 << 10]
    circ = W.Circuit(n=n, gates=gates.astype(np.int32), n_inputs=n, n_weights=single.n_weights,
                     masks=np.array(masks, np.uint64))
    x = rng.uniform(-np.pi, np.pi, size=(B, n))
    w = rng.uniform(-np.pi, np.pi, size=single.n_weights)
    G = rng.uniform(-1, 1, size=(B, len(masks)))
    got = run_gpu(circ, x, w, G, precision)
    mapped = np.array([C.heisenberg_mask(int(m), ring) for m in masks], np.uint64)
    prod = W.Circuit(n=n, gates=single.gates, n_inputs=n, n_weights=single.n_weights, masks=mapped)
    ev = np.stack([C.bloch_expvals(prod, x[b], w) for b in range(B)])
    gw = np.zeros(single.n_weights)
    gx = np.zeros((B, n))
    for b in range(B):
        gwb, gx[b] = C.bloch_grad(prod, x[b], w, G[b])
        gw += gwb
    assert_parity(got, (ev, gw, gx), precision, f"n30 {precision}")


@pytest.mark.parametrize("precision,tile,klo", [("c64", 12, 4), ("c128", 11, 4)])
def test_c5_specialised_tile_loop(precision, tile, klo):
    """n=26, 10 layers, CNOT ring, 2 samples, through the specialised kernels
    in the configurations the benchmark uses: 2^14 or 2^15 tiles per sample,
    so each workgroup loops over tiles and loads the next one during the
    current one's stages."""
    import paper_2404_06314_amd as q
    wl = W.config_workload("c5", batch=2)
    ref = fixture("oracle_c5_b2.npz")
    c = q.Circuit.from_workload(wl.circuit)
    c.set_option(q.QTM_OPT_JIT, 1)
    c.set_option(q.QTM_OPT_TILE_QUBITS, tile)
    c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=c)
    assert_parity(got, ref, precision, f"c5 specialised {precision} kt{tile}")
    # no sweep kernel spills registers to scratch memory (the complex128
    # backward kernels use up to ~350 of the 512 registers their one
    # workgroup per compute unit allows)
    for direction in (0, 1):
        for s in range(len(c.plan(precision)["sweeps"])):
            vg, sc = c.jit_info(precision, direction, s)
            assert sc <= 64, (precision, direction, s, vg, sc)
