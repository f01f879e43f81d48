"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Tolerances: complex64 <Z> 1e-5 absolute and gradients
1e-4 norm-wise relative; complex128 1e-12 and 1e-10."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import assert_parity, run_gpu

pytestmark = pytest.mark.gpu

PATHS = {"plain": 1, "fused": 2}


def _ref(wl):
    return oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("path", ["plain", "fused"])
def test_c1(precision, path):
    wl = W.config_workload("c1")
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, PATHS[path])
    assert_parity(got, _ref(wl), precision, f"c1 {path} {precision}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_c2_full_batch(precision):
    wl = W.config_workload("c2")
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision)
    assert_parity(got, _ref(wl), precision, f"c2 {precision}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,L,ent,tile,klo", [
    (6, 2, "ring", 4, 2), (9, 3, "ladder", 5, 3), (10, 2, "ring", 6, 4),
    (13, 2, "ring", 12, 5), (14, 3, "ladder", 8, 5), (11, 4, "ring", 7, 6)])
def test_multi_sweep_layered(precision, n, L, ent, tile, klo):
    rng = np.random.default_rng(n * 100 + L)
    wl = W.random_workload(rng, W.layered_circuit(n, L, ent), 3)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, 2, tile, klo)
    assert_parity(got, _ref(wl), precision, f"n{n} L{L} {ent} kt{tile}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("path", ["plain", "fused"])
def test_random_circuits(precision, path):
    rng = np.random.default_rng(77)
    for n in (4, 5, 6, 8):
        for rep in range(3):
            circ = W.random_circuit(rng, n, 60, n_inputs=3, n_weights=5, n_obs=4)
            wl = W.random_workload(rng, circ, 3)
            tile = 4 if (path == "fused" and n > 4) else None
            got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision, PATHS[path], tile, 2)
            assert_parity(got, _ref(wl), precision, f"random n{n} rep{rep} {path}")


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_circuits_use_plain_path(n):
    rng = np.random.default_rng(n)
    circ = W.random_circuit(rng, n, 12, n_inputs=2, n_weights=3, n_obs=2)
    wl = W.random_workload(rng, circ, 5)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, "c128")
    assert_parity(got, _ref(wl), "c128", f"tiny n{n}")


def test_batch_one_and_odd_batches():
    for B in (1, 3, 7):
        wl = W.config_workload("c2", batch=B)
        got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64")
        assert_parity(got, _ref(wl), "c64", f"c2 B{B}")


def test_empty_circuit_and_no_weights():
    n = 5
    circ = W.Circuit(n=n, gates=np.zeros((0, 5), np.int32), n_inputs=0, n_weights=0,
                     masks=W.z_masks(n, (0b10101,)))
    x = np.zeros((2, 0))
    got = run_gpu(circ, x, np.zeros(0), np.ones((2, circ.n_obs)), "c64")
    np.testing.assert_allclose(got[0], np.ones((2, circ.n_obs)), atol=1e-6)
    # only input-fed rotations
    c2 = W.layered_circuit(6, 2, "ring")
    g = c2.gates.copy()
    g[g[:, 3] == W.SRC_WEIGHT, 3] = W.SRC_INPUT
    g[g[:, 3] == W.SRC_INPUT, 4] %= 6
    c3 = W.Circuit(n=6, gates=g, n_inputs=6, n_weights=0, masks=c2.masks)
    rng = np.random.default_rng(3)
    wl = W.random_workload(rng, c3, 4)
    got = run_gpu(c3, wl.inputs, wl.weights, wl.grad_out, "c64")
    assert_parity(got, _ref(wl), "c64", "inputs only")


def test_recompute_and_determinism():
    import torch
    import paper_2404_06314_amd as q
    wl = W.config_workload("c2", batch=16)
    a = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64")
    b = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64")
    for u, v in zip(a, b):
        assert np.array_equal(u, v), "results differ between identical runs"
    c = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64", keep_state=False)
    for u, v in zip(a[1:], c[1:]):
        assert np.array_equal(u, v), "recomputed forward gives different gradients"


def test_state_tag_mismatch():
    import torch
    import paper_2404_06314_amd as q
    wl = W.config_workload("c1")
    c = q.Circuit.from_workload(wl.circuit)
    x = torch.as_tensor(wl.inputs, device="cuda")
    w = torch.as_tensor(wl.weights, device="cuda")
    G = torch.as_tensor(wl.grad_out, device="cuda")
    st = c.alloc_state(8, "c64")
    c.forward(x, w, "c64", state=st)
    with pytest.raises(q.QtmError) as ei:
        c.backward(x[:4].contiguous(), w, G[:4].contiguous(), "c64", state=st)
    assert ei.value.code == -5
    c.backward(x, w, G, "c64", state=st)          # matching call consumes the state
    with pytest.raises(q.QtmError):
        c.backward(x, w, G, "c64", state=st)      # consumed
    torch.cuda.synchronize()


def test_autograd_function():
    import torch
    import paper_2404_06314_amd as q
    from paper_2404_06314_amd.autograd import QtmFunction
    wl = W.config_workload("c1")
    c = q.Circuit.from_workload(wl.circuit)
    x = torch.tensor(wl.inputs, device="cuda", requires_grad=True)
    w = torch.tensor(wl.weights, device="cuda", requires_grad=True)
    out = QtmFunction.apply(x, w, c, "c128")
    G = torch.tensor(wl.grad_out, device="cuda")
    (out * G).sum().backward()
    ev, gw, gx = _ref(wl)
    np.testing.assert_allclose(out.detach().cpu().numpy(), ev, atol=1e-12)
    np.testing.assert_allclose(w.grad.cpu().numpy(), gw, atol=1e-10)
    np.testing.assert_allclose(x.grad.cpu().numpy(), gx, atol=1e-10)


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_deep_circuit_without_mid_circuit_renormalisation(precision):
    """64 layers (3584 gates) at n = 14: the complex64 state is never rescaled
    mid-circuit; the one FP64 division by the norm at the end keeps <Z> and
    the gradients within tolerance (rescaling by a scalar commutes with every
    later gate, so a periodic rescale would change only rounding)."""
    rng = np.random.default_rng(64)
    wl = W.random_workload(rng, W.layered_circuit(14, 64, "ring"), 4)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision)
    assert_parity(got, _ref(wl), precision, f"n14 L64 {precision}")


@pytest.mark.parametrize("jit", [False, True])
def test_backward_reuses_matrices_only_from_its_own_forward(jit):
    """The backward reuses the gate matrices and derivative coefficients the
    forward prepared, unless something prepared others in between: here a
    second forward with other angles into another state buffer, then the
    first buffer's backward (with its own angles), then a tile change
    between a forward and its backward.  Every result against the oracle."""
    import torch
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(1300)
    circ = W.layered_circuit(14, 3, "ladder")
    a = W.random_workload(rng, circ, 3)
    b = W.random_workload(rng, circ, 3)
    c = q.Circuit.from_workload(circ)
    if jit:
        c.set_option(q.QTM_OPT_JIT, 1)
    c.set_option(q.QTM_OPT_TILE_QUBITS, 10)
    c.set_option(q.QTM_OPT_LOW_QUBITS, 4)
    t = lambda arr: torch.as_tensor(arr, device="cuda:0")
    sa, sb = c.alloc_state(3), c.alloc_state(3)
    eva = c.forward(t(a.inputs), t(a.weights), "c64", state=sa)
    evb = c.forward(t(b.inputs), t(b.weights), "c64", state=sb)
    gwa, gxa = c.backward(t(a.inputs), t(a.weights), t(a.grad_out), "c64", state=sa)
    gwb, gxb = c.backward(t(b.inputs), t(b.weights), t(b.grad_out), "c64", state=sb)
    torch.cuda.synchronize()
    for name, wl, got in (("first", a, (eva, gwa, gxa)), ("second", b, (evb, gwb, gxb))):
        assert_parity(tuple(x.cpu().numpy() for x in got), _ref(wl), "c64", f"interleaved {name}")
    ev = c.forward(t(a.inputs), t(a.weights), "c64", state=sa)
    c.set_option(q.QTM_OPT_TILE_QUBITS, 11)
    gw, gx = c.backward(t(a.inputs), t(a.weights), t(a.grad_out), "c64", state=sa)
    torch.cuda.synchronize()
    assert_parity((ev.cpu().numpy(), gw.cpu().numpy(), gx.cpu().numpy()), _ref(a), "c64", "tile change")
