"""qtm_forward_noalloc (the forward for callers that cannot allocate) through
the C ABI: on two calls in a row, the second with a smaller batch, its
expectation values and final states equal those of qtm_forward on the same
inputs (same kernels, so bit for bit; the parity bar of 1e-5 / 1e-12 on <Z>
is asserted as well), for the compiled and the specialised sweep kernels,
the per-gate path and complex128; oversized batches and circuits whose tables
are not on the device yet are refused."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _c_forward(fn, c, B, prec, x, w, out, st):
    import torch
    P = ctypes.c_void_p
    return fn(c.handle, B, prec, P(x.data_ptr()), P(w.data_ptr()), P(out.data_ptr()),
              P(st.data_ptr()), P(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("n,ent,kind,prec", [(14, "ladder", "generic", 0), (14, "ladder", "jit", 0),
                                             (12, "ring", "jit", 1), (3, "ring", "plain", 0),
                                             (10, "ring", "generic", 1)])
def test_noalloc_forward_matches_qtm_forward(n, ent, kind, prec):
    import torch
    import paper_2404_06314_amd as q
    lib = q._lib.load()
    circ = W.layered_circuit(n, 3, ent, extra_masks=((1 << n) - 1,))
    wl = W.random_workload(np.random.default_rng(70 + n), circ, 12)
    c = q.Circuit.from_workload(circ)
    if kind == "jit":
        c.set_option(q.QTM_OPT_JIT, 1)
    dev = torch.device("cuda:0")
    tol = 1e-5 if prec == 0 else 1e-12
    for B in (12, 5):  # the second call with a smaller input
        x = torch.as_tensor(wl.inputs[:B], device=dev)
        w = torch.as_tensor(wl.weights, device=dev)
        ref = torch.empty((B, circ.n_obs), dtype=torch.float64, device=dev)
        st_ref = c.alloc_state(B, prec)
        q._lib.check(_c_forward(lib.qtm_forward, c, B, prec, x, w, ref, st_ref))
        got = torch.full((B, circ.n_obs), float("nan"), dtype=torch.float64, device=dev)
        st = torch.zeros_like(st_ref)
        q._lib.check(_c_forward(lib.qtm_forward_noalloc, c, B, prec, x, w, got, st))
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.max(np.abs(g - r)) <= tol, f"B={B}: {np.max(np.abs(g - r))}"
        assert np.array_equal(g, r)
        assert torch.equal(st, st_ref)


def test_noalloc_refusals():
    import torch
    import paper_2404_06314_amd as q
    lib = q._lib.load()
    circ = W.layered_circuit(8, 2, "ring")
    c = q.Circuit.from_workload(circ)
    dev = torch.device("cuda:0")
    B = 4
    x = torch.zeros((B, circ.n_inputs), dtype=torch.float64, device=dev)
    w = torch.zeros((circ.n_weights,), dtype=torch.float64, device=dev)
    out = torch.empty((B, circ.n_obs), dtype=torch.float64, device=dev)
    st = c.alloc_state(B, 0)
    # tables not on the device yet
    assert _c_forward(lib.qtm_forward_noalloc, c, B, 0, x, w, out, st) == q._lib.QTM_ERR_STATE
    q._lib.check(_c_forward(lib.qtm_forward, c, B, 0, x, w, out, st))
    assert _c_forward(lib.qtm_forward_noalloc, c, B, 0, x, w, out, st) == q._lib.QTM_OK
    # a batch whose buffers exceed the 16 MiB scratch (matrices alone: 64 B
    # per block and sample) is refused before anything is launched
    big = 1 << 17
    xb = torch.zeros((big, circ.n_inputs), dtype=torch.float64, device=dev)
    ob = torch.empty((big, circ.n_obs), dtype=torch.float64, device=dev)
    sb = torch.empty(8, dtype=torch.uint8, device=dev)  # never touched: refused first
    assert _c_forward(lib.qtm_forward_noalloc, c, big, 0, xb, w, ob, sb) == q._lib.QTM_ERR_WORKSPACE
    assert b"maximum" in lib.qtm_last_error()
    torch.cuda.synchronize()
