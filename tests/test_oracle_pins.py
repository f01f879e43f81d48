"""Pins for the CPU oracle: it is checked against facts fixed by the paper and
by the mathematics, never against itself.

Every pin uses a route to the numbers that is independent of the oracle's
code (see ``checkers.py``): closed forms, brute-force Kronecker unitaries,
Heisenberg propagation of Z strings, classical bit circuits, the exact
parameter-shift rule and finite differences (which use only the oracle's
forward against its reverse sweep), and invariants.
"""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
import workloads as W
import checkers as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def circ_from(d):
    gates = np.array(d["gates"], dtype=np.int32).reshape(-1, 5)
    return W.Circuit(n=d["n"], gates=gates, n_inputs=len(d["inputs"]),
                     n_weights=len(d["weights"]),
                     masks=np.array(d["masks"], dtype=np.uint64))


# --- golden closed forms ---------------------------------------------------

def test_golden_closed_forms():
    cases = json.load(open(os.path.join(GOLDEN, "closed_forms.json")))["cases"]
    for d in cases:
        c = circ_from(d)
        x = np.array(d["inputs"], dtype=float).reshape(1, -1)
        w = np.array(d["weights"], dtype=float)
        ev = oracle.forward(c, x, w)[0]
        np.testing.assert_allclose(ev, d["expect"], atol=1e-13, err_msg=d["name"])
        if "G" in d:
            _, gw, gx = oracle.vjp(c, x, w, np.array(d["G"]).reshape(1, -1))
            if "grad_w" in d:
                np.testing.assert_allclose(gw, d["grad_w"], atol=1e-13, err_msg=d["name"])
            if "grad_x" in d:
                np.testing.assert_allclose(gx[0], d["grad_x"], atol=1e-13, err_msg=d["name"])


def test_batch_split_rule():
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))["batch_split"]
    for case in facts["cases"]:
        ranges = oracle.split(case["B"], case["T"])
        assert [hi - lo for lo, hi in ranges] == case["sizes"]
        # contiguous cover of 0..B-1
        assert ranges[0][0] == 0 and ranges[-1][1] == case["B"]
        assert all(ranges[i][1] == ranges[i + 1][0] for i in range(len(ranges) - 1))


@pytest.mark.parametrize("t", [W.RX, W.RY])
def test_single_qubit_cos_and_sin(t):
    th = np.linspace(-3.0, 3.0, 13)
    c = W.Circuit(n=1, gates=np.array([[t, 0, 0, W.SRC_WEIGHT, 0]], np.int32),
                  n_inputs=0, n_weights=1, masks=np.array([1], np.uint64))
    for v in th:
        ev = oracle.forward(c, np.zeros((1, 0)), np.array([v]))[0, 0]
        assert abs(ev - math.cos(v)) < 1e-14
        _, gw, _ = oracle.vjp(c, np.zeros((1, 0)), np.array([v]), np.ones((1, 1)))
        assert abs(gw[0] + math.sin(v)) < 1e-14


def test_rz_leaves_z_unchanged_and_has_zero_gradient():
    g = np.array([[W.RY, 0, 0, W.SRC_WEIGHT, 0], [W.RZ, 0, 0, W.SRC_WEIGHT, 1]], np.int32)
    c = W.Circuit(n=1, gates=g, n_inputs=0, n_weights=2, masks=np.array([1], np.uint64))
    for a, b in [(0.3, 1.1), (-2.0, 0.7)]:
        ev = oracle.forward(c, np.zeros((1, 0)), np.array([a, b]))[0, 0]
        assert abs(ev - math.cos(a)) < 1e-14
        _, gw, _ = oracle.vjp(c, np.zeros((1, 0)), np.array([a, b]), np.ones((1, 1)))
        assert abs(gw[1]) < 1e-15


# --- product states: Bloch closed form -------------------------------------

@pytest.mark.parametrize("n,L", [(3, 1), (5, 3), (7, 2)])
def test_product_states_match_bloch(n, L):
    rng = np.random.default_rng(7 + n)
    c = W.layered_circuit(n, L, "none")
    extra = rng.integers(1, 1 << n, size=4, dtype=np.uint64)
    c.masks = np.concatenate([c.masks, extra])
    x = rng.uniform(-np.pi, np.pi, size=(3, n))
    w = rng.uniform(-np.pi, np.pi, size=c.n_weights)
    G = rng.uniform(-1, 1, size=(3, c.n_obs))
    ev, gw, gx = oracle.vjp(c, x, w, G)
    gw_ref = np.zeros_like(gw)
    for b in range(3):
        np.testing.assert_allclose(ev[b], C.bloch_expvals(c, x[b], w), atol=1e-13)
        gwb, gxb = C.bloch_grad(c, x[b], w, G[b])
        gw_ref += gwb
        np.testing.assert_allclose(gx[b], gxb, atol=1e-12)
    np.testing.assert_allclose(gw, gw_ref, atol=1e-12)


def test_one_layer_products_of_cosines():
    """One layer of RX(x) RY(w) (RZ adds only a phase): <Z_q> = cos x_q cos w_q."""
    n = 6
    rng = np.random.default_rng(3)
    c = W.layered_circuit(n, 1, "none")
    x = rng.uniform(-np.pi, np.pi, size=(2, n))
    w = rng.uniform(-np.pi, np.pi, size=c.n_weights)
    ev = oracle.forward(c, x, w)
    np.testing.assert_allclose(ev, np.cos(x) * np.cos(w[:n])[None, :], atol=1e-13)


# --- brute force (n <= 5) ----------------------------------------------------

@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 5), ng=st.integers(0, 25))
def test_brute_force_random_circuits(seed, n, ng):
    rng = np.random.default_rng(seed)
    c = W.random_circuit(rng, n, ng)
    wl = W.random_workload(rng, c, 2)
    for b in range(2):
        psi = oracle.state(c, wl.inputs[b], wl.weights)
        np.testing.assert_allclose(psi, C.brute_state(c, wl.inputs[b], wl.weights), atol=1e-12)
    ev = oracle.forward(c, wl.inputs, wl.weights)
    for b in range(2):
        np.testing.assert_allclose(ev[b], C.brute_expvals(c, wl.inputs[b], wl.weights), atol=1e-12)


def test_brute_force_config_c1():
    wl = W.config_workload("c1")
    ev = oracle.forward(wl.circuit, wl.inputs, wl.weights)
    for b in range(wl.batch):
        np.testing.assert_allclose(ev[b], C.brute_expvals(wl.circuit, wl.inputs[b], wl.weights),
                                   atol=1e-12)


# --- Heisenberg propagation: pins the CNOT ring order ----------------------

@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_ring_heisenberg(n):
    rng = np.random.default_rng(100 + n)
    c = W.layered_circuit(n, 1, "ring")
    x = rng.uniform(-np.pi, np.pi, size=(2, n))
    w = rng.uniform(-np.pi, np.pi, size=c.n_weights)
    ev = oracle.forward(c, x, w)
    rot = W.layered_circuit(n, 1, "none")
    cnots = [(int(g[1]), int(g[2])) for g in c.gates if g[0] == W.CNOT]
    assert cnots[-1] == (n - 1, 0)
    for b in range(2):
        masks = [C.heisenberg_mask(int(m), cnots) for m in c.masks]
        ref = C.bloch_expvals(rot, x[b], w, masks=masks)
        np.testing.assert_allclose(ev[b], ref, atol=1e-13)
        # the reversed ring order gives different masks (n >= 2), so the pin bites
        if n >= 3:
            masks_rev = [C.heisenberg_mask(int(m), list(reversed(cnots))) for m in c.masks]
            assert masks_rev != masks


# --- classical circuits: angles in {0, pi} --------------------------------

@pytest.mark.parametrize("n,L,ent", [(4, 3, "ring"), (9, 2, "ring"), (6, 2, "ladder")])
def test_classical_circuits(n, L, ent):
    rng = np.random.default_rng(n * 10 + L)
    c = W.layered_circuit(n, L, ent)
    x = rng.integers(0, 2, size=(3, n)) * np.pi
    w = rng.integers(-1, 2, size=c.n_weights) * np.pi
    ev = oracle.forward(c, x, w)
    for b in range(3):
        bits = C.classical_bits(c, x[b], w)
        ref = [(-1.0) ** bin(bits & int(m)).count("1") for m in c.masks]
        np.testing.assert_allclose(ev[b], ref, atol=1e-12)


# --- norm, uncompute --------------------------------------------------------

def test_norm_and_uncompute():
    wl = W.config_workload("c2", batch=2)
    for b in range(2):
        psi = oracle.state(wl.circuit, wl.inputs[b], wl.weights)
        assert abs(np.vdot(psi, psi).real - 1) < 1e-12
        assert abs(oracle.uncompute_residual(wl.circuit, wl.inputs[b], wl.weights) - 1) < 1e-10


# --- parameter shift (exact) on the untied circuit -------------------------

def _param_shift_occ(c, x_b, w, G_b):
    cu, vals, occ = C.untie(c, x_b, w)
    xb = np.asarray(x_b).reshape(1, -1)
    out = np.zeros(len(occ))
    for k in range(len(occ)):
        vp, vm = vals.copy(), vals.copy()
        vp[k] += np.pi / 2
        vm[k] -= np.pi / 2
        fp = oracle.forward(cu, xb, vp)[0]
        fm = oracle.forward(cu, xb, vm)[0]
        out[k] = np.dot(G_b, (fp - fm) / 2)
    return out, occ


@pytest.mark.parametrize("name,n,L,ent", [("c1", 4, 2, "ring"), ("lad", 5, 2, "ladder")])
def test_param_shift_per_occurrence(name, n, L, ent):
    if name == "c1":
        wl = W.config_workload("c1", batch=3)
    else:
        rng = np.random.default_rng(5)
        wl = W.random_workload(rng, W.layered_circuit(n, L, ent), 3)
    c = wl.circuit
    _, gw, gx, gocc = oracle.vjp(c, wl.inputs, wl.weights, wl.grad_out, occurrences=True)
    for b in range(wl.batch):
        ps, occ = _param_shift_occ(c, wl.inputs[b], wl.weights, wl.grad_out[b])
        np.testing.assert_allclose(gocc[b, occ], ps, atol=1e-10)


def test_param_shift_random_gates():
    rng = np.random.default_rng(11)
    for n in (2, 3, 4):
        c = W.random_circuit(rng, n, 18)
        wl = W.random_workload(rng, c, 2)
        _, _, _, gocc = oracle.vjp(c, wl.inputs, wl.weights, wl.grad_out, occurrences=True)
        for b in range(2):
            ps, occ = _param_shift_occ(c, wl.inputs[b], wl.weights, wl.grad_out[b])
            np.testing.assert_allclose(gocc[b, occ], ps, atol=1e-10)


def test_param_shift_c2_sample():
    """Exactness at n = 12 on a sample of occurrences of the c2 circuit."""
    wl = W.config_workload("c2", batch=1)
    c = wl.circuit
    _, _, _, gocc = oracle.vjp(c, wl.inputs, wl.weights, wl.grad_out, occurrences=True)
    cu, vals, occ = C.untie(c, wl.inputs[0], wl.weights)
    rng = np.random.default_rng(0)
    for k in rng.choice(len(occ), size=8, replace=False):
        vp, vm = vals.copy(), vals.copy()
        vp[k] += np.pi / 2
        vm[k] -= np.pi / 2
        fp = oracle.forward(cu, wl.inputs[:1], vp)[0]
        fm = oracle.forward(cu, wl.inputs[:1], vm)[0]
        assert abs(gocc[0, occ[k]] - np.dot(wl.grad_out[0], (fp - fm) / 2)) < 1e-10


# --- central finite differences on tied parameters --------------------------

def test_finite_differences_tied():
    wl = W.config_workload("c1", batch=4)
    c, x, w, G = wl.circuit, wl.inputs, wl.weights, wl.grad_out
    _, gw, gx = oracle.vjp(c, x, w, G)
    h = 1e-6
    L = lambda xx, ww: float(np.sum(G * oracle.forward(c, xx, ww)))
    for j in range(c.n_weights):
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        assert abs((L(x, wp) - L(x, wm)) / (2 * h) - gw[j]) < 1e-8
    for b in range(2):
        for i in range(c.n_inputs):
            xp, xm = x.copy(), x.copy()
            xp[b, i] += h
            xm[b, i] -= h
            assert abs((L(xp, w) - L(xm, w)) / (2 * h) - gx[b, i]) < 1e-8


# --- Jacobian (paper's multi-observable extension) vs VJP -----------------

def test_jacobian_rows_and_vjp_linearity():
    wl = W.config_workload("c1", batch=3)
    c = wl.circuit
    ev_j, jw, jx = oracle.jacobian(c, wl.inputs, wl.weights)
    ev_v, gw, gx = oracle.vjp(c, wl.inputs, wl.weights, wl.grad_out)
    np.testing.assert_allclose(ev_j, ev_v, atol=1e-15)
    np.testing.assert_allclose(np.einsum("bm,bmj->j", wl.grad_out, jw), gw, atol=1e-12)
    np.testing.assert_allclose(np.einsum("bm,bmi->bi", wl.grad_out, jx), gx, atol=1e-12)
    assert jw.shape == (3, c.n_obs, c.n_weights)     # (B, M, |Theta|), Sec. II-B
    # one-hot G reproduces a Jacobian row (VJP linearity)
    for m in range(c.n_obs):
        G = np.zeros((3, c.n_obs))
        G[:, m] = 1
        _, gwm, gxm = oracle.vjp(c, wl.inputs, wl.weights, G)
        np.testing.assert_allclose(gwm, jw[:, m, :].sum(0), atol=1e-12)
        np.testing.assert_allclose(gxm, jx[:, m, :], atol=1e-12)


# --- invariants ----------------------------------------------------------------

@pytest.mark.parametrize("ent", ["ring", "ladder"])
def test_last_layer_rz_gradient_is_zero(ent):
    n, L = 5, 3
    rng = np.random.default_rng(21)
    wl = W.random_workload(rng, W.layered_circuit(n, L, ent), 2)
    _, gw, _ = oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out)
    last_rz = [(L - 1) * 2 * n + n + q for q in range(n)]
    assert np.max(np.abs(gw[last_rz])) < 1e-13
    assert np.max(np.abs(gw)) > 1e-3


def test_appending_cz_layer_and_2pi_shift():
    n, L = 5, 2
    rng = np.random.default_rng(22)
    wl = W.random_workload(rng, W.layered_circuit(n, L, "ring"), 2)
    c = wl.circuit
    ev = oracle.forward(c, wl.inputs, wl.weights)
    extra = np.array([[W.CZ, i, (i + 2) % n, 0, 0] for i in range(n)], np.int32)
    c2 = W.Circuit(n=n, gates=np.concatenate([c.gates, extra]), n_inputs=c.n_inputs,
                   n_weights=c.n_weights, masks=c.masks)
    np.testing.assert_allclose(oracle.forward(c2, wl.inputs, wl.weights), ev, atol=1e-13)
    w2 = wl.weights.copy()
    w2[3] += 2 * np.pi
    np.testing.assert_allclose(oracle.forward(c, wl.inputs, w2), ev, atol=1e-12)


def test_cz_ladder_reflection_symmetry():
    n, L = 6, 2
    rng = np.random.default_rng(23)
    wl = W.random_workload(rng, W.layered_circuit(n, L, "ladder"), 2)
    c, x, w, G = wl.circuit, wl.inputs, wl.weights, wl.grad_out
    perm = np.arange(n)[::-1]
    xr = x[:, perm]
    wr = w.reshape(L, 2, n)[:, :, perm].reshape(-1)
    Gr = G[:, perm]
    ev, gw, gx = oracle.vjp(c, x, w, G)
    evr, gwr, gxr = oracle.vjp(c, xr, wr, Gr)
    np.testing.assert_allclose(evr, ev[:, perm], atol=1e-12)
    np.testing.assert_allclose(gxr, gx[:, perm], atol=1e-12)
    np.testing.assert_allclose(gwr, gw.reshape(L, 2, n)[:, :, perm].reshape(-1), atol=1e-12)


def test_amplitude_parallel_mode_matches_batch_mode():
    wl = W.config_workload("c2", batch=3)
    a = oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out, threads=4, par_mode=0)
    b = oracle.vjp(wl.circuit, wl.inputs, wl.weights, wl.grad_out, threads=4, par_mode=1)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, atol=1e-12)


# --- trainable input scaling (Sec. III-A, Eq. (7)): angle lambda * s ---------

@pytest.mark.parametrize("t", [W.RX, W.RY])
def test_scaled_single_qubit_closed_form(t):
    """RX/RY(lambda s) on |0>: <Z> = cos(lambda s); by the chain rule
    d/dlambda = -s sin(lambda s) and d/ds = -lambda sin(lambda s)."""
    c = W.Circuit(n=1, gates=np.array([[t, 0, 0, W.SRC_SCALED, 0]], np.int32),
                  n_inputs=1, n_weights=1, masks=np.array([1], np.uint64))
    for lam in (-1.3, 0.4, 1.0, 2.2):
        for s in (-2.5, -0.3, 0.0, 0.9, 3.0):
            x, w, G = np.array([[s]]), np.array([lam]), np.array([[0.7]])
            ev, gw, gx = oracle.vjp(c, x, w, G)
            assert abs(ev[0, 0] - math.cos(lam * s)) < 1e-14
            assert abs(gw[0] - 0.7 * (-s * math.sin(lam * s))) < 1e-14
            assert abs(gx[0, 0] - 0.7 * (-lam * math.sin(lam * s))) < 1e-14


def test_scaled_product_states_match_bloch():
    """Entangler-free circuits mixing plain and scaled angles: Bloch-vector
    closed form and its analytic chain-rule gradient."""
    rng = np.random.default_rng(11)
    n, n_in, n_w = 4, 3, 5
    g = []
    for _ in range(18):
        t, q = int(rng.integers(0, 3)), int(rng.integers(0, n))
        r = rng.random()
        if r < 0.5:
            g.append((t, q, int(rng.integers(0, n_w)), W.SRC_SCALED, int(rng.integers(0, n_in))))
        elif r < 0.75:
            g.append((t, q, 0, W.SRC_WEIGHT, int(rng.integers(0, n_w))))
        else:
            g.append((t, q, 0, W.SRC_INPUT, int(rng.integers(0, n_in))))
    c = W.Circuit(n=n, gates=np.array(g, np.int32), n_inputs=n_in, n_weights=n_w,
                  masks=np.array([1, 2, 4, 8, 5, 15], np.uint64))
    x = rng.uniform(-np.pi, np.pi, size=(3, n_in))
    w = rng.uniform(-1.5, 1.5, size=n_w)
    G = rng.uniform(-1, 1, size=(3, c.n_obs))
    ev, gw, gx = oracle.vjp(c, x, w, G)
    gw_ref = np.zeros_like(gw)
    for b in range(3):
        np.testing.assert_allclose(ev[b], C.bloch_expvals(c, x[b], w), atol=1e-13)
        gwb, gxb = C.bloch_grad(c, x[b], w, G[b])
        gw_ref += gwb
        np.testing.assert_allclose(gx[b], gxb, atol=1e-12)
    np.testing.assert_allclose(gw, gw_ref, atol=1e-12)


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 5), ng=st.integers(1, 25))
def test_scaled_brute_force_random_circuits(seed, n, ng):
    rng = np.random.default_rng(seed)
    c = W.random_circuit(rng, n, ng, scaled=0.5)
    wl = W.random_workload(rng, c, 2)
    ev = oracle.forward(c, wl.inputs, wl.weights)
    for b in range(2):
        np.testing.assert_allclose(ev[b], C.brute_expvals(c, wl.inputs[b], wl.weights), atol=1e-12)


def test_paper_ansatz_parameter_count():
    f = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))["ansatz_parameters"]
    c = W.paper_ansatz(f["n"], f["depth"])
    assert c.n_weights == f["count"]
    # linear in n and in d (Sec. III-A)
    assert W.paper_ansatz(6, 3).n_weights * 2 == c.n_weights
    assert W.paper_ansatz(12, 7).n_weights - W.paper_ansatz(12, 3).n_weights == 4 * 4 * 12


@pytest.mark.parametrize("ent", ["chain", "ring"])
def test_paper_ansatz_finite_differences(ent):
    """Central differences of the forward pass (no reverse sweep involved)
    against the adjoint VJP, for theta, lambda and the data inputs."""
    wl = W.paper_workload(4, 2, batch=3, seed=5, entangler=ent)
    c, x, w, G = wl.circuit, wl.inputs, wl.weights, wl.grad_out
    _, gw, gx = oracle.vjp(c, x, w, G)
    h = 1e-6
    L = lambda xx, ww: float(np.sum(G * oracle.forward(c, xx, ww)))
    for j in range(c.n_weights):
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        assert abs((L(x, wp) - L(x, wm)) / (2 * h) - gw[j]) < 1e-8, j
    for b in range(3):
        for i in range(c.n_inputs):
            xp, xm = x.copy(), x.copy()
            xp[b, i] += h
            xm[b, i] -= h
            assert abs((L(xp, w) - L(xm, w)) / (2 * h) - gx[b, i]) < 1e-8, (b, i)


def test_paper_ansatz_brute_force_and_jacobian():
    """The ansatz state against the Kronecker-product unitary, and every row of
    the Jacobian against the VJP with a one-hot upstream gradient."""
    wl = W.paper_workload(4, 2, batch=2, seed=9)
    c, x, w = wl.circuit, wl.inputs, wl.weights
    ev = oracle.forward(c, x, w)
    for b in range(2):
        np.testing.assert_allclose(ev[b], C.brute_expvals(c, x[b], w), atol=1e-12)
    _, jw, jx = oracle.jacobian(c, x, w)
    for m in range(c.n_obs):
        Gm = np.zeros((2, c.n_obs))
        Gm[:, m] = 1.0
        _, gw, gx = oracle.vjp(c, x, w, Gm)
        np.testing.assert_allclose(jw[:, m, :].sum(axis=0), gw, atol=1e-12)
        np.testing.assert_allclose(jx[:, m, :], gx, atol=1e-12)


# --- Pauli-string observables with X and Y factors ---------------------------

def test_pauli_single_qubit_closed_forms():
    """RY(t)|0> has Bloch vector (sin t, 0, cos t); RX(t)|0> has (0, -sin t, cos t)."""
    for t_type, want_x, want_y in ((W.RY, math.sin, lambda t: 0.0),
                                   (W.RX, lambda t: 0.0, lambda t: -math.sin(t))):
        c = W.with_observables(
            W.Circuit(n=1, gates=np.array([[t_type, 0, 0, W.SRC_WEIGHT, 0]], np.int32),
                      n_inputs=0, n_weights=1, masks=np.array([1], np.uint64)),
            [{0: "X"}, {0: "Y"}, {0: "Z"}])
        for t in (-2.7, -0.4, 0.0, 1.1, 2.9):
            ev, gw, _ = oracle.vjp(c, np.zeros((1, 0)), np.array([t]), np.array([[1.0, 0.0, 0.0]]))
            np.testing.assert_allclose(ev[0], [want_x(t), want_y(t), math.cos(t)], atol=1e-14)
            h = 1e-6
            assert abs(gw[0] - (want_x(t + h) - want_x(t - h)) / (2 * h)) < 1e-8
            _, gw, _ = oracle.vjp(c, np.zeros((1, 0)), np.array([t]), np.array([[0.0, 1.0, 0.0]]))
            assert abs(gw[0] - (want_y(t + h) - want_y(t - h)) / (2 * h)) < 1e-8


def test_pauli_bell_state():
    """RY(pi/2) then CNOT(0 -> 1) makes (|00> + |11>) / sqrt 2: <XX> = 1,
    <YY> = -1, <ZZ> = 1, <XY> = <X_0> = <Y_1> = 0."""
    c = W.with_observables(
        W.Circuit(n=2, gates=np.array([[W.RY, 0, 0, W.SRC_WEIGHT, 0], [W.CNOT, 0, 1, 0, 0]], np.int32),
                  n_inputs=0, n_weights=1, masks=np.array([1], np.uint64)),
        [{0: "X", 1: "X"}, {0: "Y", 1: "Y"}, {0: "Z", 1: "Z"}, {0: "X", 1: "Y"}, {0: "X"}, {1: "Y"}])
    ev = oracle.forward(c, np.zeros((1, 0)), np.array([math.pi / 2]))
    np.testing.assert_allclose(ev[0], [1, -1, 1, 0, 0, 0], atol=1e-14)


def test_pauli_product_states_match_bloch():
    rng = np.random.default_rng(19)
    n = 5
    base = W.layered_circuit(n, 2, "none")
    c = W.with_observables(base, W.random_pauli_strings(rng, n, 12, max_weight=4))
    x = rng.uniform(-np.pi, np.pi, size=(3, n))
    w = rng.uniform(-np.pi, np.pi, size=c.n_weights)
    G = rng.uniform(-1, 1, size=(3, c.n_obs))
    ev, gw, gx = oracle.vjp(c, x, w, G)
    gw_ref = np.zeros_like(gw)
    for b in range(3):
        np.testing.assert_allclose(ev[b], C.bloch_expvals(c, x[b], w), atol=1e-13)
        gwb, gxb = C.bloch_grad(c, x[b], w, G[b])
        gw_ref += gwb
        np.testing.assert_allclose(gx[b], gxb, atol=1e-12)
    np.testing.assert_allclose(gw, gw_ref, atol=1e-12)


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 5), ng=st.integers(0, 25))
def test_pauli_brute_force_random_circuits(seed, n, ng):
    rng = np.random.default_rng(seed)
    c = W.with_observables(W.random_circuit(rng, n, ng), W.random_pauli_strings(rng, n, 4))
    wl = W.random_workload(rng, c, 2)
    ev = oracle.forward(c, wl.inputs, wl.weights)
    for b in range(2):
        np.testing.assert_allclose(ev[b], C.brute_expvals(c, wl.inputs[b], wl.weights), atol=1e-12)


def test_pauli_finite_differences_and_jacobian():
    """Entangled circuit, mixed Z / X / Y strings: the adjoint VJP against
    central differences of the forward, and every Jacobian row against the
    VJP with a one-hot upstream gradient."""
    rng = np.random.default_rng(23)
    c = W.with_observables(W.layered_circuit(4, 3, "ring"),
                           [{0: "Z"}, {1: "X"}, {2: "Y", 3: "X"}, {0: "Y", 1: "Z", 3: "Y"}, {3: "Z", 0: "Z"}])
    wl = W.random_workload(rng, c, 3)
    x, w, G = wl.inputs, wl.weights, wl.grad_out
    _, gw, gx = oracle.vjp(c, x, w, G)
    h = 1e-6
    L = lambda xx, ww: float(np.sum(G * oracle.forward(c, xx, ww)))
    for j in range(c.n_weights):
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        assert abs((L(x, wp) - L(x, wm)) / (2 * h) - gw[j]) < 1e-8, j
    for i in range(c.n_inputs):
        xp, xm = x.copy(), x.copy()
        xp[1, i] += h
        xm[1, i] -= h
        assert abs((L(xp, w) - L(xm, w)) / (2 * h) - gx[1, i]) < 1e-8, i
    _, jw, jx = oracle.jacobian(c, x, w)
    for m in range(c.n_obs):
        Gm = np.zeros((3, c.n_obs))
        Gm[:, m] = 1.0
        _, gwm, gxm = oracle.vjp(c, x, w, Gm)
        np.testing.assert_allclose(jw[:, m, :].sum(axis=0), gwm, atol=1e-12)
        np.testing.assert_allclose(jx[:, m, :], gxm, atol=1e-12)


# --- fixed one-qubit gates and controlled rotations --------------------------

def _circ(n, gates, n_inputs=0, n_weights=1, strings=None):
    c = W.Circuit(n=n, gates=np.array(gates, np.int32).reshape(-1, 5), n_inputs=n_inputs,
                  n_weights=n_weights, masks=np.array([1], np.uint64))
    return W.with_observables(c, strings) if strings else c


def test_fixed_gate_closed_forms():
    """Textbook facts: H|0> = |+>, S H|0> = |+i>, T T = S, X and Y flip Z,
    SX SX = X, Z H|0> = |->."""
    none = np.zeros((1, 0))
    w = np.zeros(1)
    axes = [{0: "X"}, {0: "Y"}, {0: "Z"}]
    cases = [
        ([[W.H, 0, 0, 0, 0]], [1, 0, 0]),
        ([[W.H, 0, 0, 0, 0], [W.S, 0, 0, 0, 0]], [0, 1, 0]),
        ([[W.H, 0, 0, 0, 0], [W.SDG, 0, 0, 0, 0]], [0, -1, 0]),
        ([[W.H, 0, 0, 0, 0], [W.T, 0, 0, 0, 0], [W.T, 0, 0, 0, 0]], [0, 1, 0]),
        ([[W.H, 0, 0, 0, 0], [W.TDG, 0, 0, 0, 0], [W.TDG, 0, 0, 0, 0]], [0, -1, 0]),
        ([[W.H, 0, 0, 0, 0], [W.T, 0, 0, 0, 0]], [math.sqrt(0.5), math.sqrt(0.5), 0]),
        ([[W.X, 0, 0, 0, 0]], [0, 0, -1]),
        ([[W.Y, 0, 0, 0, 0]], [0, 0, -1]),
        ([[W.SX, 0, 0, 0, 0], [W.SX, 0, 0, 0, 0]], [0, 0, -1]),
        ([[W.SX, 0, 0, 0, 0]], [0, -1, 0]),
        ([[W.H, 0, 0, 0, 0], [W.Z, 0, 0, 0, 0]], [-1, 0, 0]),
    ]
    for gates, want in cases:
        ev = oracle.forward(_circ(1, gates, strings=axes), none, w)
        np.testing.assert_allclose(ev[0], want, atol=1e-14, err_msg=str(gates))


def test_controlled_rotation_closed_forms():
    """CRY(t) with the control in |1>: <Z_t> = cos t; control in |0>: 1 and no
    gradient; control in |+> (H): (1 + cos t) / 2 with derivative -sin t / 2.
    CRZ(t) between |+> states: <X_t> = (1 + cos t) / 2 (the target's Bloch
    vector turns by t about z where the control is 1)."""
    for t in (-2.2, -0.5, 0.3, 1.7, 3.0):
        w = np.array([t])
        z1 = [{1: "Z"}]
        ev = oracle.forward(_circ(2, [[W.X, 0, 0, 0, 0], [W.CRY, 0, 1, W.SRC_WEIGHT, 0]], strings=z1),
                            np.zeros((1, 0)), w)
        assert abs(ev[0, 0] - math.cos(t)) < 1e-14
        ev, gw, _ = oracle.vjp(_circ(2, [[W.CRY, 0, 1, W.SRC_WEIGHT, 0]], strings=z1),
                               np.zeros((1, 0)), w, np.ones((1, 1)))
        assert abs(ev[0, 0] - 1) < 1e-14 and abs(gw[0]) < 1e-15
        ev, gw, _ = oracle.vjp(_circ(2, [[W.H, 0, 0, 0, 0], [W.CRY, 0, 1, W.SRC_WEIGHT, 0]], strings=z1),
                               np.zeros((1, 0)), w, np.ones((1, 1)))
        assert abs(ev[0, 0] - (1 + math.cos(t)) / 2) < 1e-14
        assert abs(gw[0] + math.sin(t) / 2) < 1e-14
        ev, gw, _ = oracle.vjp(_circ(2, [[W.H, 0, 0, 0, 0], [W.H, 1, 0, 0, 0],
                                         [W.CRZ, 0, 1, W.SRC_WEIGHT, 0]], strings=[{1: "X"}]),
                               np.zeros((1, 0)), w, np.ones((1, 1)))
        assert abs(ev[0, 0] - (1 + math.cos(t)) / 2) < 1e-14
        assert abs(gw[0] + math.sin(t) / 2) < 1e-14


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(1, 5), ng=st.integers(0, 30))
def test_extended_gates_brute_force(seed, n, ng):
    rng = np.random.default_rng(seed)
    c = W.with_observables(W.random_circuit(rng, n, ng, extended=0.5), W.random_pauli_strings(rng, n, 3))
    wl = W.random_workload(rng, c, 2)
    for b in range(2):
        psi = oracle.state(c, wl.inputs[b], wl.weights)
        np.testing.assert_allclose(psi, C.brute_state(c, wl.inputs[b], wl.weights), atol=1e-12)
    ev = oracle.forward(c, wl.inputs, wl.weights)
    for b in range(2):
        np.testing.assert_allclose(ev[b], C.brute_expvals(c, wl.inputs[b], wl.weights), atol=1e-12)


def test_extended_gates_finite_differences():
    """Random circuits with fixed gates and controlled rotations (parameters
    shared between gates): the adjoint VJP against central differences."""
    rng = np.random.default_rng(71)
    for n in (2, 4, 5):
        c = W.with_observables(W.random_circuit(rng, n, 40, n_inputs=3, n_weights=4, extended=0.5),
                               W.random_pauli_strings(rng, n, 3))
        wl = W.random_workload(rng, c, 2)
        x, w, G = wl.inputs, wl.weights, wl.grad_out
        _, gw, gx = oracle.vjp(c, x, w, G)
        h = 1e-6
        L = lambda xx, ww: float(np.sum(G * oracle.forward(c, xx, ww)))
        for j in range(c.n_weights):
            wp, wm = w.copy(), w.copy()
            wp[j] += h
            wm[j] -= h
            assert abs((L(x, wp) - L(x, wm)) / (2 * h) - gw[j]) < 1e-8, (n, j)
        for i in range(c.n_inputs):
            xp, xm = x.copy(), x.copy()
            xp[0, i] += h
            xm[0, i] -= h
            assert abs((L(xp, w) - L(xm, w)) / (2 * h) - gx[0, i]) < 1e-8, (n, i)
