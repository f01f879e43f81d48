"""GPU parity for weight-scaled input angles (trainable input scaling of the
paper's ansatz, Sec. III-A Eq. (7)): the paper's benchmark shapes (Fig. 1:
n = 4..18, B = 48, d = 3, M = n; Fig. 2: n = 12, B = 48, d = 1..11), random
circuits mixing plain and scaled angles with shared slots, the Jacobian, the
specialised (JIT) sweeps and the uneven-batch runtime, each against the
oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import FLOOR_G_C64, TOL_G_C64, TOL_Z_C64, assert_grad_close, assert_parity, run_gpu

pytestmark = pytest.mark.gpu


def _ref(wl):
    return oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)


@pytest.mark.parametrize("n,B", [(4, 48), (8, 48), (12, 48), (16, 48), (18, 4)])
def test_fig1_qubit_sweep(n, B):
    wl = W.paper_workload(n, 3, B, seed=300 + n)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64")
    assert_parity(got, _ref(wl), "c64", f"paper n{n} d3 B{B}")


@pytest.mark.parametrize("d", [1, 6, 11])
def test_fig2_depth_sweep(d):
    wl = W.paper_workload(12, d, 48, seed=400 + d)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64")
    assert_parity(got, _ref(wl), "c64", f"paper n12 d{d}")


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("path,tile,klo", [(1, None, None), (2, None, None), (2, 5, 2)])
def test_paths_and_precisions(precision, path, tile, klo):
    wl = W.paper_workload(9, 3, 6, seed=17, entangler="ring")
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, path, tile, klo)
    assert_parity(got, _ref(wl), precision, f"paper n9 ring path{path} kt{tile}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("path", [1, 2])
def test_random_scaled_circuits(precision, path):
    rng = np.random.default_rng(2024)
    for n in (4, 6, 9):
        for rep in range(3):
            circ = W.random_circuit(rng, n, 70, n_inputs=3, n_weights=4, n_obs=3, scaled=0.5)
            wl = W.random_workload(rng, circ, 3)
            tile = 4 if (path == 2 and n > 4) else None
            got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision, path, tile, 2)
            assert_parity(got, _ref(wl), precision, f"random scaled n{n} rep{rep} path{path}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("n,d", [(10, 3), (12, 3), (12, 6)])
def test_jit_single_tile_samples(precision, n, d):
    """One sweep with a workgroup per sample (tile = n): the specialised
    forward prepares its sample's gate matrices and derivative coefficients
    (weight-scaled input angles included) and the backward writes the
    per-rotation gradients, without the prep and slot-reduction launches."""
    import paper_2404_06314_amd as q
    wl = W.paper_workload(n, d, 6, seed=700 + 10 * n + d)
    c = q.Circuit.from_workload(wl.circuit)
    c.set_option(q.QTM_OPT_JIT, 1)
    c.set_option(q.QTM_OPT_TILE_QUBITS, n)
    assert len(c.plan(precision)["sweeps"]) == 1
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=c)
    assert_parity(got, _ref(wl), precision, f"paper n{n} d{d} jit single tile {precision}")


def test_jit_sweeps():
    import paper_2404_06314_amd as q
    wl = W.paper_workload(14, 3, 8, seed=23)
    c = q.Circuit.from_workload(wl.circuit)
    c.set_option(q.QTM_OPT_JIT, 1)
    got = run_gpu(wl.circuit, wl.inputs, wl.weights, wl.grad_out, "c64", qcirc=c)
    assert_parity(got, _ref(wl), "c64", "paper n14 d3 jit")


@pytest.mark.parametrize("precision,jit", [("c64", False), ("c128", False), ("c64", True), ("c128", True)])
def test_jacobian(precision, jit):
    """The Jacobian of the paper's ansatz (10 qubits, depth 2); with the
    specialised sweeps the plan is one sweep over single-tile samples, whose
    kernels prepare the gates and write the per-rotation gradients
    themselves."""
    import torch
    import paper_2404_06314_amd as q
    from gpu_helpers import FLOOR_G_C128, TOL_G_C128, TOL_Z_C128
    wl = W.paper_workload(10, 2, 4, seed=31)
    c = q.Circuit.from_workload(wl.circuit)
    if jit:
        c.set_option(q.QTM_OPT_JIT, 1)
        assert len(c.plan(precision)["sweeps"]) == 1
    xt = torch.as_tensor(wl.inputs, dtype=torch.float64, device="cuda:0")
    wt = torch.as_tensor(wl.weights, dtype=torch.float64, device="cuda:0")
    ev, jw, jx = c.jacobian(xt, wt, precision)
    torch.cuda.synchronize()
    rev, rjw, rjx = oracle.jacobian(wl.circuit, wl.inputs, wl.weights)
    tz, tg, fl = ((TOL_Z_C64, TOL_G_C64, FLOOR_G_C64) if precision == "c64"
                  else (TOL_Z_C128, TOL_G_C128, FLOOR_G_C128))
    assert np.max(np.abs(ev.cpu().numpy() - rev)) <= tz
    jw, jx = jw.cpu().numpy(), jx.cpu().numpy()
    for b in range(4):
        for m in range(wl.circuit.n_obs):
            assert_grad_close(jw[b, m], rjw[b, m], tg, f"J_w[{b},{m}]", fl)
            assert_grad_close(jx[b, m], rjx[b, m], tg, f"J_x[{b},{m}]", fl)


def test_uneven_batch_of_paper_circuits():
    """Persistent uneven-batch kernels over paper-ansatz items of 2..14 qubits
    and depth 1..5 (items below 4 qubits take the per-gate path)."""
    import torch
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(41)
    items = []
    for i in range(24):
        n = int(rng.integers(2, 15))
        d = int(rng.integers(1, 6))
        items.append(W.paper_workload(n, d, 1, seed=1000 + i))
    m = q.Multi([q.Circuit.from_workload(wl.circuit) for wl in items])
    cat = lambda arrs: np.concatenate([a.reshape(-1) for a in arrs])
    x, w, G = (torch.as_tensor(cat(a), dtype=torch.float64, device="cuda:0")
               for a in ([wl.inputs for wl in items], [wl.weights for wl in items],
                         [wl.grad_out for wl in items]))
    st = m.alloc_state()
    ev = m.forward(x, w, st)
    gw, gx = m.backward(x, w, G, st)
    torch.cuda.synchronize()
    ev, gw, gx = ev.cpu().numpy(), gw.cpu().numpy(), gx.cpu().numpy()
    for i, wl in enumerate(items):
        rev, rgw, rgx = _ref(wl)
        e = ev[m.out_off[i]:m.out_off[i + 1]]
        assert np.max(np.abs(e - rev[0])) <= TOL_Z_C64, f"item {i}"
        assert_grad_close(gw[m.w_off[i]:m.w_off[i + 1]], rgw, TOL_G_C64, f"item {i} dL/dw", FLOOR_G_C64)
        assert_grad_close(gx[m.in_off[i]:m.in_off[i + 1]], rgx[0], TOL_G_C64, f"item {i} dL/dx",
                          FLOOR_G_C64)
