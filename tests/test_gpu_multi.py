"""Uneven batch: many circuits of different width and depth, one sample each,
run by the persistent kernels (graph-launched) through qtm_multi_*; every
checked item is compared with the oracle run on that item alone."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import workloads as W
from gpu_helpers import FLOOR_G_C64, TOL_G_C64, TOL_Z_C64, assert_grad_close, report

pytestmark = pytest.mark.gpu


def oracle_items(items):
    import oracle

    def one(wl):
        ev, gw, gx = oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out, threads=1)
        return ev[0], gw, gx[0]

    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, items))


def packed(items):
    x = np.concatenate([wl.inputs.reshape(-1) for wl in items] + [np.zeros(0)])
    w = np.concatenate([wl.weights.reshape(-1) for wl in items] + [np.zeros(0)])
    G = np.concatenate([wl.grad_out.reshape(-1) for wl in items] + [np.zeros(0)])
    return x, w, G


def to_dev(*arrs):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
            for a in arrs]


def run_multi(m, items, arrays=None):
    import torch
    x, w, G = to_dev(*(arrays or packed(items)))
    st = m.alloc_state()
    ev = m.forward(x, w, st)
    gw, gx = m.backward(x, w, G, st)
    torch.cuda.synchronize()
    return ev.cpu().numpy(), gw.cpu().numpy(), gx.cpu().numpy()


def check_items(m, got, refs, which, what=""):
    ev, gw, gx = got
    ez = rw = rx = 0.0
    for i, (rev, rgw, rgx) in zip(which, refs):
        e = ev[m.out_off[i]:m.out_off[i + 1]]
        err = np.max(np.abs(e - rev))
        assert err <= TOL_Z_C64, f"{what} item {i}: <Z> err {err:.3e}"
        ez = max(ez, err)
        rw = max(rw, assert_grad_close(gw[m.w_off[i]:m.w_off[i + 1]], rgw, TOL_G_C64,
                                       f"{what} item {i} dL/dw", FLOOR_G_C64))
        rx = max(rx, assert_grad_close(gx[m.in_off[i]:m.in_off[i + 1]], rgx, TOL_G_C64,
                                       f"{what} item {i} dL/dx", FLOOR_G_C64))
    report(f"{what} ({len(refs)} items)", z_abs=ez, gw_rel=rw, gx_rel=rx)


def mixed_items(seed=7):
    """Layered circuits of 4..14 qubits (ring, CZ ladder, no entangler), random
    circuits with shared parameter slots and several observables, and narrow
    circuits of 1..3 qubits that take the per-gate path."""
    rng = np.random.default_rng(seed)
    out = []
    for k, (n, L, ent) in enumerate([(4, 1, "ring"), (5, 3, "ladder"), (8, 2, "ring"),
                                     (9, 4, "none"), (11, 3, "ladder"), (12, 2, "ring"),
                                     (13, 2, "ring"), (14, 1, "ladder"), (6, 4, "ring"),
                                     (12, 10, "ring"), (7, 1, "ladder")]):
        circ = W.layered_circuit(n, L, ent, extra_masks=((1 << n) - 1,) if k % 2 else ())
        out.append(W.random_workload(rng, circ, 1))
    for n, g in [(4, 30), (6, 60), (9, 80), (13, 50)]:
        out.append(W.random_workload(rng, W.random_circuit(rng, n, g), 1))
    for n in (1, 2, 3):
        out.append(W.random_workload(rng, W.random_circuit(rng, n, 8), 1))
    order = rng.permutation(len(out))
    return [out[i] for i in order]


def make_multi(items):
    import paper_2404_06314_amd as q
    return q.Multi([q.Circuit.from_workload(wl.circuit) for wl in items])


def test_mixed_items_against_oracle():
    items = mixed_items()
    m = make_multi(items)
    got = run_multi(m, items)
    check_items(m, got, oracle_items(items), range(len(items)), "mixed")


def test_units_cover_every_tile():
    import paper_2404_06314_amd as q
    items = mixed_items()
    m = make_multi(items)
    run_multi(m, items)
    want = 0
    for wl in items:
        c = wl.circuit
        if c.n < 4:
            continue
        plan = q.Circuit.from_workload(c).plan("c64")
        want += len(plan["sweeps"]) * (1 << (c.n - plan["kt"]))
    assert m.units(0) == want and m.units(1) == want


def test_graph_replays_and_pointer_updates():
    """Three calls through the same graphs with fresh input tensors (so the
    graph nodes' pointers are patched), eager torch work in between; each
    against the oracle, and against the eagerly launched kernels (timing
    mode) bit for bit."""
    import torch
    base = mixed_items(11)
    m = make_multi(base)
    rng = np.random.default_rng(5)
    for rep in range(3):
        items = [W.random_workload(rng, wl.circuit, 1) for wl in base]
        got = run_multi(m, items)
        junk = torch.randn(1 << 20, device="cuda:0")
        (junk * 2).sum().item()
        check_items(m, got, oracle_items(items), range(len(items)), f"replay {rep}")
        m.set_timing(True)
        eager = run_multi(m, items)
        m.timing_read(0)
        m.timing_read(1)
        m.set_timing(False)
        for a, b in zip(got, eager):
            assert np.array_equal(a, b)


def test_repeat_is_bitwise_identical():
    items = W.uneven_items(48, seed=99)
    m = make_multi(items)
    a = run_multi(m, items)
    b = run_multi(m, items)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_uneven_1024_full_launch():
    """The 1024-circuit uneven batch (n 8..16, 2..10 layers, CNOT ring) in the
    launch bench.py times: every item against the oracle run on that item
    alone."""
    items = W.uneven_items(1024)
    m = make_multi(items)
    got = run_multi(m, items)
    ev, gw, gx = got
    assert np.all(np.isfinite(ev)) and np.all(np.isfinite(gw)) and np.all(np.isfinite(gx))
    check_items(m, got, oracle_items(items), range(len(items)), "uneven1024")
