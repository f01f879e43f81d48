"""GPU parity for fixed one-qubit gates (H, X, Y, Z, S, S^dag, T, T^dag, SX:
fused into the per-wire blocks) and controlled rotations (CRX, CRY, CRZ: the
per-gate path), against the oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import FLOOR_G_C64, TOL_G_C64, TOL_Z_C64, assert_grad_close, assert_parity, run_gpu

pytestmark = pytest.mark.gpu


def _ref(wl):
    return oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)


def _fixed_only(rng, n, n_gates):
    """Random circuit with fixed gates but no controlled rotation."""
    while True:
        c = W.random_circuit(rng, n, n_gates, n_inputs=3, n_weights=5, extended=0.4)
        keep = [int(t) not in W.CONTROLLED_TYPES for t in c.gates[:, 0]]
        g = c.gates[keep]
        if any(int(t) in W.FIXED_TYPES for t in g[:, 0]):
            return W.Circuit(n=n, gates=g, n_inputs=3, n_weights=5, masks=c.masks)


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("path,tile", [(1, None), (2, None), (2, 4)])
def test_fixed_gates(precision, path, tile):
    rng = np.random.default_rng(55)
    for n in (4, 6, 9):
        circ = W.with_observables(_fixed_only(rng, n, 70), W.random_pauli_strings(rng, n, 4))
        wl = W.random_workload(rng, circ, 3)
        t = tile if (tile and n > tile) else None
        got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision, path, t, 2 if t else None)
        assert_parity(got, _ref(wl), precision, f"fixed n{n} path{path} tile{t}")


def test_fixed_gates_specialised_sweeps():
    """A 14-qubit layered circuit with Hadamard, S and T layers between the
    rotation layers, through the specialised sweeps."""
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(14)
    base = W.layered_circuit(14, 3, "ring")
    extra = []
    for l, gates in enumerate(np.split(base.gates, 3)):
        extra.extend(gates.tolist())
        extra.extend([[W.H if l % 2 == 0 else W.SX, q_, 0, 0, 0] for q_ in range(14)])
        extra.extend([[W.T, q_, 0, 0, 0] for q_ in range(0, 14, 2)])
        extra.extend([[W.SDG, q_, 0, 0, 0] for q_ in range(1, 14, 3)])
    circ = W.Circuit(n=14, gates=np.array(extra, np.int32), n_inputs=base.n_inputs,
                     n_weights=base.n_weights, masks=base.masks)
    wl = W.random_workload(rng, circ, 6)
    c = q.Circuit.from_workload(circ)
    c.set_option(q.QTM_OPT_JIT, 1)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, "c64", qcirc=c)
    assert_parity(got, _ref(wl), "c64", "n14 fixed layers jit")


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_controlled_rotations(precision):
    rng = np.random.default_rng(66)
    for n in (2, 3, 5, 8, 10):
        circ = W.with_observables(W.random_circuit(rng, n, 60, n_inputs=3, n_weights=5, extended=0.5),
                                  W.random_pauli_strings(rng, n, 4))
        wl = W.random_workload(rng, circ, 3)
        got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision)
        assert_parity(got, _ref(wl), precision, f"controlled n{n}")


def test_controlled_rotations_refuse_the_fused_path():
    import torch
    import paper_2404_06314_amd as q
    circ = W.Circuit(n=5, gates=np.array([[W.CRX, 0, 3, W.SRC_WEIGHT, 0]], np.int32), n_inputs=0,
                     n_weights=1, masks=np.array([8], np.uint64))
    c = q.Circuit.from_workload(circ)
    c.set_path(q.QTM_PATH_FUSED)
    x = torch.zeros((2, 0), dtype=torch.float64, device="cuda:0")
    w = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(q.QtmError) as ei:
        c.forward(x, w, "c64")
    assert ei.value.code == -2


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_jacobian_with_controlled_rotations(precision):
    import torch
    import paper_2404_06314_amd as q
    from gpu_helpers import FLOOR_G_C128, TOL_G_C128, TOL_Z_C128
    rng = np.random.default_rng(77)
    circ = W.with_observables(W.random_circuit(rng, 6, 50, n_inputs=3, n_weights=4, extended=0.5),
                              W.random_pauli_strings(rng, 6, 3))
    wl = W.random_workload(rng, circ, 3)
    c = q.Circuit.from_workload(circ)
    ev, jw, jx = c.jacobian(torch.as_tensor(wl.inputs, device="cuda:0"),
                            torch.as_tensor(wl.weights, device="cuda:0"), precision)
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


def test_uneven_batch_with_new_gates():
    """Items with fixed gates run in the persistent kernels; items with
    controlled rotations run one by one."""
    import torch
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(88)
    items = []
    for i in range(12):
        n = int(rng.integers(3, 11))
        circ = _fixed_only(rng, n, 40) if i % 3 else W.random_circuit(rng, n, 40, extended=0.5)
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
