"""GPU parity for circuits whose qubits are excited late.  The state starts
at |0...0>, so until a qubit meets its first non-diagonal gate (a rotation
block that is not diagonal, or a CNOT target) every amplitude with its bit
set is 0; the specialised sweeps skip tiles and loads of such amplitudes and
keep only what later sweeps read.  These circuits excite qubits one group at
a time, by rotations and by CNOT targets, put diagonal blocks and CZs on
qubits before their first rotation, leave a qubit unexcited to the end
(with X and Y observables on it), and run through the matrix-core kernels
with one tile per workgroup and with a tile loop, and through the
complex128 kernels; each against the oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import assert_parity, run_gpu

pytestmark = pytest.mark.gpu


def staircase(n: int, layers: int, step: int, idle=(), strings=None) -> W.Circuit:
    """Layer l rotates qubits below (l + 1) * step (RX input, RY and RZ
    weights) and applies a CZ ladder over them; the next qubit up gets RZ and
    a CZ to the active group (diagonal, it stays unexcited) and, every other
    layer, a CNOT from the top active qubit (which excites it).  Qubits in
    `idle` only ever get RZ and CZ."""
    g, nw = [], 0
    for l in range(layers):
        top = min(n, (l + 1) * step)
        act = [q for q in range(top) if q not in idle]
        for q in act:
            g.append([W.RX, q, 0, W.SRC_INPUT, q % 4])
            g.append([W.RY, q, 0, W.SRC_WEIGHT, nw]); nw += 1
            g.append([W.RZ, q, 0, W.SRC_WEIGHT, nw]); nw += 1
        for a, b in zip(act, act[1:]):
            g.append([W.CZ, a, b, 0, 0])
        if top < n:
            g.append([W.RZ, top, 0, W.SRC_WEIGHT, nw]); nw += 1
            g.append([W.CZ, act[-1], top, 0, 0])
            if l % 2 == 1:
                g.append([W.CNOT, act[-1], top, 0, 0])
        for q in idle:
            g.append([W.RZ, q, 0, W.SRC_WEIGHT, nw]); nw += 1
            g.append([W.CZ, q, (q + 1) % n, 0, 0])
    circ = W.Circuit(n=n, gates=np.array(g, np.int32), n_inputs=4, n_weights=nw,
                     masks=W.z_masks(n, extra=((1 << n) - 1,)))
    return W.with_observables(circ, strings) if strings else circ


def _run(circ, B, seed, precision, tile, klo):
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(seed)
    wl = W.random_workload(rng, circ, B)
    c = q.Circuit.from_workload(circ)
    c.set_option(q.QTM_OPT_JIT, 1)
    c.set_option(q.QTM_OPT_TILE_QUBITS, tile)
    c.set_option(q.QTM_OPT_LOW_QUBITS, klo)
    got = run_gpu(circ, wl.inputs, wl.weights, wl.grad_out, precision, qcirc=c)
    ref = oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)
    return c, got, ref


def _plan_has_dead_sweeps(c, precision):
    """At least one sweep before the last leaves some qubit unexcited."""
    p = c.plan(precision)
    full = (1 << p["n"]) - 1
    return any(e != full for e in p["excited"][:-1])


@pytest.mark.parametrize("n,tile,klo,step,layers", [(16, 10, 4, 3, 6), (16, 11, 3, 4, 5),
                                                    (18, 12, 5, 5, 4), (14, 10, 4, 2, 8)])
def test_staircase_matrix_core(n, tile, klo, step, layers):
    circ = staircase(n, layers, step)
    c, got, ref = _run(circ, 3, 900 + n, "c64", tile, klo)
    assert _plan_has_dead_sweeps(c, "c64")
    assert_parity(got, ref, "c64", f"staircase n{n} kt{tile} klo{klo}")


def test_staircase_tile_loop():
    """2^(n - tile) = 1024 tiles per sample: the kernels loop over tiles."""
    circ = staircase(20, 4, 6)
    c, got, ref = _run(circ, 2, 920, "c64", 10, 4)
    assert _plan_has_dead_sweeps(c, "c64")
    assert_parity(got, ref, "c64", "staircase n20 kt10 tile loop")


@pytest.mark.parametrize("tile,klo", [(6, 3), (8, 4)])
def test_staircase_complex128(tile, klo):
    circ = staircase(12, 5, 3)
    c, got, ref = _run(circ, 3, 930 + tile, "c128", tile, klo)
    assert _plan_has_dead_sweeps(c, "c128")
    assert_parity(got, ref, "c128", f"staircase n12 c128 kt{tile}")


@pytest.mark.parametrize("precision,tile,klo", [("c64", 10, 4), ("c128", 7, 3)])
def test_qubit_never_excited(precision, tile, klo):
    """Qubit 13 gets only RZ and CZ: <X_13> and <Y_13 Z_0> are 0, but the bra
    terms of those strings are not, and live on amplitudes the sweeps take
    as 0."""
    n = 14
    strings = ([{q: "Z"} for q in range(n)] + [{13: "X"}, {13: "Y", 0: "Z"}, {12: "X", 13: "Y"},
                                              {11: "Y", 12: "X"}])
    circ = staircase(n, 5, 3, idle=(13,), strings=strings)
    c, got, ref = _run(circ, 3, 940, precision, tile, klo)
    full = (1 << n) - 1
    assert c.plan(precision)["excited"][-1] == full & ~(1 << 13)
    assert_parity(got, ref, precision, f"never excited {precision}")


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_jacobian_staircase(precision):
    """The Jacobian (one backward per observable) through the specialised
    sweeps on a circuit whose qubits are excited late."""
    import torch
    import paper_2404_06314_amd as q
    from gpu_helpers import (FLOOR_G_C64, FLOOR_G_C128, TOL_G_C64, TOL_G_C128, TOL_Z_C64, TOL_Z_C128,
                             assert_grad_close)
    circ = staircase(14, 5, 3, strings=[{0: "Z"}, {13: "X"}, {5: "Y", 6: "Z"}, {12: "Z", 13: "Z"}])
    rng = np.random.default_rng(950)
    wl = W.random_workload(rng, circ, 2)
    c = q.Circuit.from_workload(circ)
    c.set_option(q.QTM_OPT_JIT, 1)
    c.set_option(q.QTM_OPT_TILE_QUBITS, 10 if precision == "c64" else 7)
    c.set_option(q.QTM_OPT_LOW_QUBITS, 4 if precision == "c64" else 3)
    assert _plan_has_dead_sweeps(c, precision)
    ev, jw, jx = c.jacobian(torch.as_tensor(wl.inputs, device="cuda:0"),
                            torch.as_tensor(wl.weights, device="cuda:0"), precision)
    torch.cuda.synchronize()
    rev, rjw, rjx = oracle.jacobian(circ, wl.inputs, wl.weights)
    tz, tg, fl = ((TOL_Z_C64, TOL_G_C64, FLOOR_G_C64) if precision == "c64"
                  else (TOL_Z_C128, TOL_G_C128, FLOOR_G_C128))
    assert np.max(np.abs(ev.cpu().numpy() - rev)) <= tz
    jw, jx = jw.cpu().numpy(), jx.cpu().numpy()
    for b in range(2):
        for m in range(circ.n_obs):
            assert_grad_close(jw[b, m], rjw[b, m], tg, f"J_w[{b},{m}]", fl)
            assert_grad_close(jx[b, m], rjx[b, m], tg, f"J_x[{b},{m}]", fl)


def test_no_kept_state_and_recomputed_forward():
    """Forward without a kept state, then a backward that recomputes the
    forward itself, through the specialised sweeps."""
    import torch
    import paper_2404_06314_amd as q
    circ = staircase(16, 6, 3)
    rng = np.random.default_rng(960)
    wl = W.random_workload(rng, circ, 3)
    c = q.Circuit.from_workload(circ)
    c.set_option(q.QTM_OPT_JIT, 1)
    c.set_option(q.QTM_OPT_TILE_QUBITS, 10)
    c.set_option(q.QTM_OPT_LOW_QUBITS, 4)
    x, w, G = (torch.as_tensor(a, device="cuda:0") for a in (wl.inputs, wl.weights, wl.grad_out))
    ev = c.forward(x, w, "c64", state=None)
    gw, gx = c.backward(x, w, G, "c64", state=None)
    torch.cuda.synchronize()
    ref = oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)
    assert_parity((ev.cpu().numpy(), gw.cpu().numpy(), gx.cpu().numpy()), ref, "c64", "no kept state")


def test_degenerate_circuits_specialised():
    """Extremes of the zero-amplitude logic through the specialised kernels
    (14 qubits, tile 10): an empty circuit (only |0...0> is ever nonzero), a
    circuit of diagonal gates only (no qubit is ever excited; X and Y
    observables on top), and qubits excited only by fixed gates (H, X, SX)."""
    n = 14
    empty = W.Circuit(n=n, gates=np.zeros((0, 5), np.int32), n_inputs=0, n_weights=0,
                      masks=W.z_masks(n, ((1 << n) - 1,)))
    diag = []
    for q_ in range(n):
        diag.append([W.RZ, q_, 0, W.SRC_WEIGHT, q_])
        diag.append([W.S if q_ % 2 else W.T, q_, 0, 0, 0])
    diag += [[W.CZ, q_, q_ + 1, 0, 0] for q_ in range(n - 1)]
    diag_c = W.with_observables(
        W.Circuit(n=n, gates=np.array(diag, np.int32), n_inputs=0, n_weights=n, masks=W.z_masks(n)),
        [{q_: "Z"} for q_ in range(n)] + [{3: "X"}, {5: "Y", 6: "X"}, {0: "Z", 13: "Z"}])
    fixed = []
    for q_ in range(n):
        fixed.append([(W.H, W.X, W.SX)[q_ % 3], q_, 0, 0, 0])
        fixed.append([W.RZ, q_, 0, W.SRC_WEIGHT, q_])
        fixed.append([W.RY, q_, 0, W.SRC_INPUT, q_ % 2])
    fixed += [[W.CNOT, q_, (q_ + 3) % n, 0, 0] for q_ in range(n)]
    fixed_c = W.Circuit(n=n, gates=np.array(fixed, np.int32), n_inputs=2, n_weights=n, masks=W.z_masks(n))
    for name, circ in (("empty", empty), ("diagonal", diag_c), ("fixed", fixed_c)):
        c, got, ref = _run(circ, 2, 980, "c64", 10, 4)
        assert_parity(got, ref, "c64", f"degenerate {name}")
        if name == "empty":
            np.testing.assert_allclose(got[0], 1.0, atol=1e-6)
