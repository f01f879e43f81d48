"""GPU parity for observables that are Pauli strings with X and Y factors
(the paper admits any observable, Sec. II-A): expectation values, the VJP
and the Jacobian through both kernel paths, both precisions, the
specialised sweeps, forward without a kept state, backward with the
forward recomputed, and circuits with such observables inside an uneven
batch; each against the oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import FLOOR_G_C64, TOL_G_C64, TOL_Z_C64, assert_grad_close, assert_parity, run_gpu

pytestmark = pytest.mark.gpu


def _ref(wl):
    return oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)


def every_axis(n):
    return [{q: p} for q in range(n) for p in "XYZ"]


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("path", [1, 2])
def test_random_circuits_random_strings(precision, path):
    rng = np.random.default_rng(808)
    for n in (4, 5, 7, 9):
        for rep in range(2):
            circ = W.with_observables(W.random_circuit(rng, n, 60, n_inputs=3, n_weights=5, scaled=0.2),
                                      W.random_pauli_strings(rng, n, 6, max_weight=4))
            wl = W.random_workload(rng, circ, 3)
            tile = 4 if (path == 2 and n > 4) else None
            got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision, path, tile, 2)
            assert_parity(got, _ref(wl), precision, f"pauli n{n} rep{rep} path{path}")


@pytest.mark.parametrize("precision,jit", [("c64", False), ("c64", True), ("c128", False)])
def test_layered_every_axis(precision, jit):
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(12)
    circ = W.with_observables(W.layered_circuit(12, 4, "ring"),
                              every_axis(12) + [{0: "X", 5: "Y", 11: "X"}, {3: "Y", 4: "Y"}])
    wl = W.random_workload(rng, circ, 16)
    c = q.Circuit.from_workload(circ)
    if jit:
        c.set_option(q.QTM_OPT_JIT, 1)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=c)
    assert_parity(got, _ref(wl), precision, f"n12 every axis jit={jit}")


def test_n20_strings_full_size():
    """The n = 20, 8-layer CZ-ladder circuit with Z on every qubit plus X and
    Y strings, batch 4, through the default path."""
    rng = np.random.default_rng(20)
    base = W.config_workload("c3", batch=4)
    strings = [{q: "Z"} for q in range(20)] + [{0: "X"}, {19: "Y"}, {7: "X", 8: "X"}, {2: "Y", 15: "Z"}]
    circ = W.with_observables(base.circuit, strings)
    G = rng.uniform(-1, 1, size=(4, len(strings)))
    wl = W.Workload(circuit=circ, batch=4, inputs=base.inputs, weights=base.weights, grad_out=G)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, "c64")
    assert_parity(got, _ref(wl), "c64", "n20 pauli")


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_jacobian(precision):
    import torch
    import paper_2404_06314_amd as q
    from gpu_helpers import FLOOR_G_C128, TOL_G_C128, TOL_Z_C128
    rng = np.random.default_rng(31)
    circ = W.with_observables(W.paper_ansatz(8, 2), [{0: "X"}, {1: "Y"}, {2: "Z"}, {3: "X", 4: "Y"}])
    wl = W.random_workload(rng, circ, 3)
    c = q.Circuit.from_workload(circ)
    xt = torch.as_tensor(wl.inputs, device="cuda:0")
    wt = torch.as_tensor(wl.weights, device="cuda:0")
    ev, jw, jx = c.jacobian(xt, wt, precision)
    torch.cuda.synchronize()
    rev, rjw, rjx = oracle.jacobian(circ, wl.inputs, wl.weights)
    tz, tg, fl = ((TOL_Z_C64, TOL_G_C64, FLOOR_G_C64) if precision == "c64"
                  else (TOL_Z_C128, TOL_G_C128, FLOOR_G_C128))
    assert np.max(np.abs(ev.cpu().numpy() - rev)) <= tz
    jw, jx = jw.cpu().numpy(), jx.cpu().numpy()
    for b in range(3):
        for m in range(circ.n_obs):
            assert_grad_close(jw[b, m], rjw[b, m], tg, f"J_w[{b},{m}]", fl)
            assert_grad_close(jx[b, m], rjx[b, m], tg, f"J_x[{b},{m}]", fl)


def test_no_kept_state_and_recomputed_backward():
    """qtm_forward with state = NULL (final states in the workspace) and
    qtm_backward with state = NULL (forward recomputed inside)."""
    import torch
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(5)
    circ = W.with_observables(W.layered_circuit(10, 3, "ladder"), every_axis(10))
    wl = W.random_workload(rng, circ, 5)
    c = q.Circuit.from_workload(circ)
    x, w, G = (torch.as_tensor(a, device="cuda:0") for a in (wl.inputs, wl.weights, wl.grad_out))
    ev = c.forward(x, w, "c64", state=None)
    gw, gx = c.backward(x, w, G, "c64", state=None)
    torch.cuda.synchronize()
    assert_parity((ev.cpu().numpy(), gw.cpu().numpy(), gx.cpu().numpy()), _ref(wl), "c64",
                  "no kept state")


def test_uneven_batch_with_pauli_items():
    import torch
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(9)
    items = []
    for i in range(10):
        n = int(rng.integers(3, 12))
        circ = W.layered_circuit(n, int(rng.integers(1, 4)), "ring")
        if i % 3 == 0:
            circ = W.with_observables(circ, W.random_pauli_strings(rng, n, 4))
        items.append(W.random_workload(rng, circ, 1))
    m = q.Multi([q.Circuit.from_workload(wl.circuit) for wl in items])
    cat = lambda arrs: np.concatenate([a.reshape(-1) for a in arrs])
    x, w, G = (torch.as_tensor(cat(a), device="cuda:0")
               for a in ([wl.inputs for wl in items], [wl.weights for wl in items],
                         [wl.grad_out for wl in items]))
    st = m.alloc_state()
    ev = m.forward(x, w, st)
    gw, gx = m.backward(x, w, G, st)
    torch.cuda.synchronize()
    ev, gw, gx = ev.cpu().numpy(), gw.cpu().numpy(), gx.cpu().numpy()
    for i, wl in enumerate(items):
        rev, rgw, rgx = _ref(wl)
        assert np.max(np.abs(ev[m.out_off[i]:m.out_off[i + 1]] - rev[0])) <= TOL_Z_C64, f"item {i}"
        assert_grad_close(gw[m.w_off[i]:m.w_off[i + 1]], rgw, TOL_G_C64, f"item {i} dL/dw", FLOOR_G_C64)
        assert_grad_close(gx[m.in_off[i]:m.in_off[i + 1]], rgx[0], TOL_G_C64, f"item {i} dL/dx",
                          FLOOR_G_C64)
