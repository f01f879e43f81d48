"""A forward + backward step captured in a HIP graph (torch.cuda.CUDAGraph
on the library's stream argument) and replayed: after one eager call has
sized the workspaces, the entry points launch kernels only (no allocation,
no memset, no synchronisation), so the step can be captured. Every replay,
with eager calls and synchronisations between replays, must reproduce the
eager step bit for bit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,jit", [("c64", True), ("c64", False), ("c128", False)])
def test_step_replayed_from_graph(precision, jit):
    import torch
    import paper_2404_06314_amd as q
    rng = np.random.default_rng(1200)
    circ = W.layered_circuit(14, 3, "ladder")
    wl = W.random_workload(rng, circ, 4)
    c = q.Circuit.from_workload(circ)
    if jit:
        c.set_option(q.QTM_OPT_JIT, 1)
        c.set_option(q.QTM_OPT_TILE_QUBITS, 10)
        c.set_option(q.QTM_OPT_LOW_QUBITS, 4)
    dev = torch.device("cuda:0")
    x, w, G = (torch.as_tensor(a, device=dev) for a in (wl.inputs, wl.weights, wl.grad_out))
    st = c.alloc_state(4, precision)

    def step():
        ev = c.forward(x, w, precision, state=st)
        gw, gx = c.backward(x, w, G, precision, state=st)
        return ev, gw, gx

    ref = [t.clone() for t in step()]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = step()
    torch.cuda.synchronize()
    for r in range(4):
        for t in out:
            t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b), f"replay {r}"
        again = step()
        torch.cuda.synchronize()
        for a, b in zip(again, ref):
            assert torch.equal(a, b), f"eager call after replay {r}"
