"""Independent checkers used to pin the oracle.

None of these call the oracle or share its code.  Each follows a different
route to the same numbers:

* ``brute_*``: the full 2^n x 2^n unitary built from Kronecker products of
  ``scipy.linalg.expm(-i theta P / 2)`` factors (qubit 0 is the right-most
  factor), entanglers built from projector sums; observables as Kronecker
  products of Z and I.
* ``bloch_*``: entangler-free circuits stay product states; each qubit's Bloch
  vector is rotated by SO(3) matrices and <Z_S> is the product of z parts.
* ``heisenberg_mask``: a CNOT conjugates a Z string into another Z string.
* ``classical_*``: with every angle in {0, pi} the state is one basis vector
  up to a phase.
"""
from __future__ import annotations

import math
from functools import reduce

import numpy as np
import scipy.linalg as sla

import workloads as W

PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2, dtype=complex)
P0 = np.array([[1, 0], [0, 0]], dtype=complex)
P1 = np.array([[0, 0], [0, 1]], dtype=complex)
PAULI = {W.RX: PX, W.RY: PY, W.RZ: PZ}
_R2 = 1 / math.sqrt(2)
FIXED = {
    W.H: np.array([[1, 1], [1, -1]]) * _R2, W.X: PX, W.Y: PY, W.Z: PZ,
    W.S: np.diag([1, 1j]), W.SDG: np.diag([1, -1j]),
    W.T: np.diag([1, np.exp(0.25j * np.pi)]), W.TDG: np.diag([1, np.exp(-0.25j * np.pi)]),
    W.SX: sla.sqrtm(PX),
}


def kron_on(n, ops: dict):
    """Kronecker product over qubits n-1 ... 0 with ops[q] on qubit q."""
    return reduce(np.kron, [ops.get(q, I2) for q in reversed(range(n))])


def _angle(g, x_b, w):
    if g[3] == W.SRC_SCALED:
        return w[g[2]] * x_b[g[4]]
    return x_b[g[4]] if g[3] == W.SRC_INPUT else w[g[4]]


def brute_unitary(circ, x_b, w):
    n = circ.n
    U = np.eye(1 << n, dtype=complex)
    for g in circ.gates:
        t, q0, q1 = int(g[0]), int(g[1]), int(g[2])
        if t in W.PARAM_TYPES:
            th = _angle(g, x_b, w)
            G = kron_on(n, {q0: sla.expm(-0.5j * th * PAULI[t])})
        elif t in W.FIXED_TYPES:
            G = kron_on(n, {q0: FIXED[t]})
        elif t in W.CONTROLLED_TYPES:
            th = _angle(g, x_b, w)
            R = sla.expm(-0.5j * th * PAULI[t - W.CRX])
            G = kron_on(n, {q0: P0}) + kron_on(n, {q0: P1, q1: R})
        elif t == W.CNOT:
            G = kron_on(n, {q0: P0}) + kron_on(n, {q0: P1, q1: PX})
        else:
            G = np.eye(1 << n) - 2 * kron_on(n, {q0: P1, q1: P1})
        U = G @ U
    return U


def brute_state(circ, x_b, w):
    psi0 = np.zeros(1 << circ.n, dtype=complex)
    psi0[0] = 1
    return brute_unitary(circ, x_b, w) @ psi0


def zstring(n, mask):
    return kron_on(n, {q: PZ for q in range(n) if (int(mask) >> q) & 1})


def pauli_string(n, xmask, zmask):
    """Kronecker product of X, Y, Z factors: X where only the X bit is set, Z
    where only the Z bit is, Y where both are."""
    ops = {}
    for q in range(n):
        xb, zb = (int(xmask) >> q) & 1, (int(zmask) >> q) & 1
        if xb or zb:
            ops[q] = PY if (xb and zb) else (PX if xb else PZ)
    return kron_on(n, ops)


def observables(circ):
    xm = circ.xmasks if getattr(circ, "xmasks", None) is not None else np.zeros_like(circ.masks)
    return list(zip(xm, circ.masks))


def brute_expvals(circ, x_b, w):
    psi = brute_state(circ, x_b, w)
    return np.array([np.real(np.vdot(psi, pauli_string(circ.n, xm, zm) @ psi))
                     for xm, zm in observables(circ)])


# --- Bloch-vector closed forms for product states -------------------------

def so3(t, th):
    c, s = math.cos(th), math.sin(th)
    if t == W.RX:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if t == W.RY:
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def so3_deriv(t, th):
    c, s = math.cos(th), math.sin(th)
    if t == W.RX:
        return np.array([[0, 0, 0], [0, -s, -c], [0, c, -s]])
    if t == W.RY:
        return np.array([[-s, 0, c], [0, 0, 0], [-c, 0, -s]])
    return np.array([[-s, -c, 0], [c, -s, 0], [0, 0, 0]])


def bloch_vectors(circ, x_b, w):
    r = {q: np.array([0.0, 0.0, 1.0]) for q in range(circ.n)}
    for g in circ.gates:
        t = int(g[0])
        assert t in W.PARAM_TYPES, "product-state closed form needs no entangler"
        r[int(g[1])] = so3(t, _angle(g, x_b, w)) @ r[int(g[1])]
    return r


def _axis(xm, zm, q):
    """Bloch component (0 x, 1 y, 2 z) a Pauli factor on qubit q reads, or None."""
    xb, zb = (int(xm) >> q) & 1, (int(zm) >> q) & 1
    if not (xb or zb):
        return None
    return 1 if (xb and zb) else (0 if xb else 2)


def bloch_expvals(circ, x_b, w, masks=None):
    """<P> of a product state is the product over the string's factors of the
    matching Bloch components."""
    r = bloch_vectors(circ, x_b, w)
    obs = observables(circ) if masks is None else [(0, m) for m in masks]
    out = []
    for xm, zm in obs:
        out.append(np.prod([r[q][_axis(xm, zm, q)] for q in range(circ.n)
                            if _axis(xm, zm, q) is not None]))
    return np.array(out)


def bloch_grad(circ, x_b, w, G):
    """Analytic VJP of the product-state closed form (chain + product rule)."""
    n = circ.n
    per_q = {q: [] for q in range(n)}
    for k, g in enumerate(circ.gates):
        per_q[int(g[1])].append(k)
    gw = np.zeros(circ.n_weights)
    gx = np.zeros(circ.n_inputs)
    r = bloch_vectors(circ, x_b, w)
    for q in range(n):
        ks = per_q[q]
        mats = [so3(int(circ.gates[k][0]), _angle(circ.gates[k], x_b, w)) for k in ks]
        for j, k in enumerate(ks):
            v = np.array([0.0, 0.0, 1.0])
            for i, M in enumerate(mats):
                if i == j:
                    v = so3_deriv(int(circ.gates[k][0]), _angle(circ.gates[k], x_b, w)) @ v
                else:
                    v = M @ v
            tot = 0.0
            for (xm, zm), Gm in zip(observables(circ), G):
                a = _axis(xm, zm, q)
                if a is None:
                    continue
                others = np.prod([r[p][_axis(xm, zm, p)] for p in range(n)
                                  if p != q and _axis(xm, zm, p) is not None])
                tot += Gm * v[a] * others
            g = circ.gates[k]
            if g[3] == W.SRC_WEIGHT:
                gw[g[4]] += tot
            elif g[3] == W.SRC_INPUT:
                gx[g[4]] += tot
            else:  # angle w[q1] * x[idx]
                gw[g[2]] += tot * x_b[g[4]]
                gx[g[4]] += tot * w[g[2]]
    return gw, gx


# --- untied circuits: every rotation occurrence its own parameter -------

def angle_value(src: int, idx: int, q1: int, x_b: np.ndarray, w: np.ndarray) -> float:
    """The number a rotation record selects (a lookup; for a scaled input the
    product of the two slots it names)."""
    if src == W.SRC_INPUT:
        return float(x_b[idx])
    if src == W.SRC_WEIGHT:
        return float(w[idx])
    return float(w[q1]) * float(x_b[idx])


def untie(circ: W.Circuit, x: np.ndarray, w: np.ndarray):
    """Give every parameterised gate occurrence its own weight slot.

    Returns (circuit, weights, occ) where the new circuit reads every rotation
    angle from its own weight slot k (in gate order) and ``occ[k]`` is the gate
    index.  Input-fed angles are copied from the single sample ``x``.
    Used by parameter-shift checks: the shift rule is exact only for a
    parameter that enters exactly one exp(-i theta P / 2).
    """
    g = circ.gates.copy()
    vals, occ = [], []
    for k in range(g.shape[0]):
        t, q0, q1, src, idx = (int(v) for v in g[k])
        if t in W.PARAM_TYPES:
            vals.append(angle_value(src, idx, q1, x, w))
            g[k, 2] = 0
            g[k, 3] = W.SRC_WEIGHT
            g[k, 4] = len(occ)
            occ.append(k)
    c = W.Circuit(n=circ.n, gates=g, n_inputs=max(circ.n_inputs, 1),
                n_weights=len(occ), masks=circ.masks.copy(),
                name=circ.name + "_untied")
    return c, np.array(vals, dtype=np.float64), occ


def untie_to_inputs(circ: W.Circuit, x_b: np.ndarray, w: np.ndarray):
    """Like `untie`, but every rotation occurrence k reads input slot k, so a
    batch of rows can carry differently shifted angle vectors.  Returns
    (circuit, base_row, occ) with base_row[k] the angle of occurrence k."""
    g = circ.gates.copy()
    vals, occ = [], []
    for k in range(g.shape[0]):
        t, q0, q1, src, idx = (int(v) for v in g[k])
        if t in W.PARAM_TYPES:
            vals.append(angle_value(src, idx, q1, x_b, w))
            g[k, 2] = 0
            g[k, 3] = W.SRC_INPUT
            g[k, 4] = len(occ)
            occ.append(k)
    c = W.Circuit(n=circ.n, gates=g, n_inputs=len(occ), n_weights=0, masks=circ.masks.copy(),
                name=circ.name + "_untied_inputs")
    return c, np.array(vals, dtype=np.float64), occ


# --- Heisenberg propagation of Z strings through CNOTs ---------------------

def heisenberg_mask(mask: int, cnots) -> int:
    """U^dag Z_S U for U = C_N ... C_1 (C_1 applied first): conjugate by the
    last gate first.  CNOT(c, t): Z_t -> Z_c Z_t, Z_c -> Z_c."""
    s = int(mask)
    for c, t in reversed(list(cnots)):
        if (s >> t) & 1:
            s ^= 1 << c
    return s


# --- classical circuits ----------------------------------------------------

def classical_bits(circ, x_b, w):
    """Angles must be 0 or pi (mod 2 pi): RX(pi), RY(pi) flip a bit, RZ only
    adds a phase, CNOT permutes, CZ adds a sign."""
    bits = 0
    for g in circ.gates:
        t, q0, q1 = int(g[0]), int(g[1]), int(g[2])
        if t in (W.RX, W.RY):
            th = _angle(g, x_b, w)
            k = round(th / math.pi)
            assert abs(th - k * math.pi) < 1e-12
            if k % 2:
                bits ^= 1 << q0
        elif t == W.CNOT:
            if (bits >> q0) & 1:
                bits ^= 1 << q1
    return bits
