"""Diagnostics and guards of the C ABI: the per-sample state norms of the last
forward (norm-drift watchdog), the optional non-finite angle check, and the
workspace cap that makes QTM_ERR_WORKSPACE reachable."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _setup(n, L, ent, B, seed=3):
    import torch
    circ = W.layered_circuit(n, L, ent)
    wl = W.random_workload(np.random.default_rng(seed), circ, B)
    dev = torch.device("cuda:0")
    return circ, wl, torch.as_tensor(wl.inputs, device=dev), torch.as_tensor(wl.weights, device=dev), \
        torch.as_tensor(wl.grad_out, device=dev)


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,kind", [(3, "plain"), (8, "generic"), (8, "jit"), (10, "jit-single-tile"),
                                    (14, "jit"), (14, "plain")])
def test_forward_norms_match_the_states(precision, n, kind):
    """qtm_forward_norms returns each sample's squared norm from the forward's
    own reduction: equal to the norm of the kept final state (summed here in
    float64 by torch) and within the precision's drift of 1."""
    import torch
    import paper_2404_06314_amd as q
    circ, wl, x, w, G = _setup(n, 3, "ring", 5)
    c = q.Circuit.from_workload(circ)
    if kind == "plain":
        c.set_path(q.QTM_PATH_PLAIN)
    if kind.startswith("jit"):
        c.set_option(q.QTM_OPT_JIT, 1)
    if kind == "jit-single-tile":
        c.set_option(q.QTM_OPT_TILE_QUBITS, n)
    st = c.alloc_state(5, precision)
    c.forward(x, w, precision, state=st)
    nr = c.forward_norms(5).cpu().numpy()
    cdt = torch.complex64 if precision == "c64" else torch.complex128
    amps = st.view(cdt).view(5, 1 << n)
    ref = (amps.real.double() ** 2 + amps.imag.double() ** 2).sum(dim=1).cpu().numpy()
    # the library sums each thread's 16 probabilities in the state's precision
    # (FP64 from there on), the reference everything in FP64
    assert np.max(np.abs(nr - ref)) <= (2e-6 if precision == "c64" else 1e-13) * np.max(ref)
    drift = 1e-5 if precision == "c64" else 1e-12
    assert np.max(np.abs(nr - 1.0)) <= drift
    with pytest.raises(q.QtmError) as e:
        c.forward_norms(4)
    assert e.value.code == -5


def test_forward_norms_after_a_per_gate_backward_is_refused():
    import paper_2404_06314_amd as q
    circ, wl, x, w, G = _setup(6, 2, "ring", 3)
    c = q.Circuit.from_workload(circ)
    c.set_path(q.QTM_PATH_PLAIN)
    st = c.alloc_state(3, "c64")
    c.forward(x, w, "c64", state=st)
    c.forward_norms(3)
    c.backward(x, w, G, "c64", state=st)
    with pytest.raises(q.QtmError) as e:
        c.forward_norms(3)
    assert e.value.code == -5


@pytest.mark.parametrize("path", ["fused", "plain"])
def test_non_finite_angles_are_rejected(path):
    """With QTM_OPT_CHECK_ANGLES a NaN or infinity in the inputs or weights is
    an error naming the entry, for the forward, the backward and the
    Jacobian; finite values give the same results as without the check."""
    import torch
    import paper_2404_06314_amd as q
    circ, wl, x, w, G = _setup(8, 2, "ladder", 4)
    c = q.Circuit.from_workload(circ)
    c.set_path(q.QTM_PATH_FUSED if path == "fused" else q.QTM_PATH_PLAIN)
    ref = c.forward(x, w, "c64").cpu().numpy()
    c.set_option(q.QTM_OPT_CHECK_ANGLES, 1)
    got = c.forward(x, w, "c64").cpu().numpy()
    assert np.array_equal(ref, got)
    xb = x.clone()
    xb[1, 2] = float("nan")
    with pytest.raises(q.QtmError) as e:
        c.forward(xb, w, "c64")
    assert e.value.code == -1 and "inputs[1][2]" in str(e.value)
    wb = w.clone()
    wb[3] = float("inf")
    with pytest.raises(q.QtmError) as e:
        c.backward(x, wb, G, "c64")
    assert e.value.code == -1 and "weights[3]" in str(e.value)
    with pytest.raises(q.QtmError) as e:
        c.jacobian(xb, w, "c64")
    assert e.value.code == -1
    c.set_option(q.QTM_OPT_CHECK_ANGLES, 0)
    torch.cuda.synchronize()


def test_workspace_cap():
    """QTM_MAX_WORKSPACE_BYTES bounds a handle's device workspace: a forward
    that would need more returns QTM_ERR_WORKSPACE; a value that is not a
    byte count is refused the same way; without the cap the call works."""
    import paper_2404_06314_amd as q
    circ, wl, x, w, G = _setup(10, 2, "ring", 4)
    old = os.environ.get("QTM_MAX_WORKSPACE_BYTES")
    try:
        os.environ["QTM_MAX_WORKSPACE_BYTES"] = "4096"
        c = q.Circuit.from_workload(circ)
        with pytest.raises(q.QtmError) as e:
            c.forward(x, w, "c64")  # state = NULL: a 32 KiB state workspace
        assert e.value.code == -3 and "QTM_MAX_WORKSPACE_BYTES" in str(e.value)
        os.environ["QTM_MAX_WORKSPACE_BYTES"] = "lots"
        with pytest.raises(q.QtmError) as e:
            c.forward(x, w, "c64")
        assert e.value.code == -3
        os.environ["QTM_MAX_WORKSPACE_BYTES"] = str(1 << 30)
        c.forward(x, w, "c64")
    finally:
        if old is None:
            os.environ.pop("QTM_MAX_WORKSPACE_BYTES", None)
        else:
            os.environ["QTM_MAX_WORKSPACE_BYTES"] = old


def test_layer_drift_watchdog():
    """QuantumLayer(drift_tol=...) reads the forward's state norms: the drift of
    a complex64 forward stays below 1e-5, and a tolerance below it warns."""
    import warnings

    import torch
    import paper_2404_06314_amd as q
    from paper_2404_06314_amd.autograd import QuantumLayer
    circ = W.layered_circuit(10, 3, "ring")
    layer = QuantumLayer(q.Circuit.from_workload(circ), "c64", drift_tol=1e-5)
    x = torch.rand((4, circ.n_inputs), dtype=torch.float64, device="cuda")
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        layer(x)
    assert 0.0 <= layer.last_drift <= 1e-5
    layer.drift_tol = 0.0
    if layer.last_drift > 0.0:
        with pytest.warns(RuntimeWarning):
            layer(x)
