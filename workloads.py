"""Seeded synthetic inputs: circuits (gate lists), angles, upstream gradients.

This module is the only code shared by the oracle side and the HIP side.  It
holds none of the method's arithmetic: it emits gate *records* (which gate,
on which qubits, reading which input or weight slot), observable bitmasks and
random numbers, and nothing that simulates a state.

Gate record format (int32 x 5): ``type, q0, q1, src, index``.

* ``type``: 0 RX, 1 RY, 2 RZ, 3 CNOT (q0 = control, q1 = target), 4 CZ;
  fixed one-qubit gates on q0: 5 H, 6 X, 7 Y, 8 Z, 9 S, 10 S^dag, 11 T,
  12 T^dag, 13 SX; controlled rotations 14 CRX, 15 CRY, 16 CRZ (q0 =
  control, q1 = target, src 1 or 2).
* ``src``: 0 none (entanglers), 1 input vector, 2 weight vector, 3 weight-
  scaled input: angle ``weights[q1] * inputs[index]`` (the trainable input
  scaling lambda * s of the paper's ansatz, Sec. III-A Eq. (7)).
* ``index``: slot in that vector.  Parameters are indexed in construction
  order, never alphabetically (paper Sec. II-C).

Circuit family (paper Eq. (7), simplified to the layer used by every
benchmark here): one *layer* is RX(x_q) angle encoding on each qubit
(re-uploaded every layer, Sec. III-A "data re-uploading"), then trainable RY
and RZ on each qubit, then an entangler: a CNOT ring i -> (i+1) mod n applied
in increasing i (wrap gate last), or an open CZ ladder (i, i+1).  Weight slot
``l*2n + q`` is the RY angle on qubit q in layer l, ``l*2n + n + q`` the RZ
angle.  Observables are Pauli-Z strings given as bitmasks (bit q = qubit q,
little-endian basis index).

Random draws use ``numpy.random.default_rng(seed)`` in a fixed order:
weights, then inputs (row-major), then the upstream gradient G.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RX, RY, RZ, CNOT, CZ = 0, 1, 2, 3, 4
H, X, Y, Z, S, SDG, T, TDG, SX = 5, 6, 7, 8, 9, 10, 11, 12, 13
CRX, CRY, CRZ = 14, 15, 16
FIXED_TYPES = (H, X, Y, Z, S, SDG, T, TDG, SX)
CONTROLLED_TYPES = (CRX, CRY, CRZ)
SRC_NONE, SRC_INPUT, SRC_WEIGHT, SRC_SCALED = 0, 1, 2, 3
PARAM_TYPES = (RX, RY, RZ)


@dataclass
class Circuit:
    n: int
    gates: np.ndarray          # int32 [G, 5]
    n_inputs: int
    n_weights: int
    masks: np.ndarray          # uint64 [M]: Z-parts of the observables' Pauli strings
    name: str = ""
    xmasks: np.ndarray | None = None  # uint64 [M]: X-parts (None: every observable a Z string)

    @property
    def n_gates(self) -> int:
        return int(self.gates.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.masks.shape[0])


@dataclass
class Workload:
    circuit: Circuit
    batch: int
    inputs: np.ndarray         # float64 [B, n_inputs]
    weights: np.ndarray        # float64 [n_weights]
    grad_out: np.ndarray       # float64 [B, M]
    meta: dict = field(default_factory=dict)


def pauli(ops: dict) -> tuple[int, int]:
    """(X-part, Z-part) bitmasks of the Pauli string with factor ops[q] in
    {"X", "Y", "Z"} on qubit q (identity elsewhere): X sets the X bit, Z the
    Z bit, Y both."""
    xm = zm = 0
    for q, p in ops.items():
        if p not in ("X", "Y", "Z"):
            raise ValueError(p)
        if p in ("X", "Y"):
            xm |= 1 << int(q)
        if p in ("Y", "Z"):
            zm |= 1 << int(q)
    return xm, zm


def with_observables(circ: Circuit, strings) -> Circuit:
    """The same circuit with the given observables (a list of ops dicts for
    `pauli`)."""
    xz = [pauli(o) for o in strings]
    return Circuit(n=circ.n, gates=circ.gates, n_inputs=circ.n_inputs, n_weights=circ.n_weights,
                   masks=np.array([z for _, z in xz], dtype=np.uint64),
                   xmasks=np.array([x for x, _ in xz], dtype=np.uint64),
                   name=circ.name + "_pauli")


def random_pauli_strings(rng, n: int, count: int, max_weight: int = 3):
    """Random Pauli strings (ops dicts) of weight 1..max_weight."""
    out = []
    for _ in range(count):
        k = int(rng.integers(1, min(max_weight, n) + 1))
        qs = rng.choice(n, size=k, replace=False)
        out.append({int(q): "XYZ"[int(rng.integers(0, 3))] for q in qs})
    return out


def z_masks(n: int, extra=()) -> np.ndarray:
    """Single-qubit Z_i on every qubit, then any extra masks."""
    return np.array([1 << q for q in range(n)] + list(extra), dtype=np.uint64)


def layered_circuit(n: int, layers: int, entangler: str = "ring",
                    extra_masks=(), name: str = "") -> Circuit:
    if entangler not in ("ring", "ladder", "none"):
        raise ValueError(entangler)
    g = []
    for l in range(layers):
        for q in range(n):
            g.append((RX, q, 0, SRC_INPUT, q))
        for q in range(n):
            g.append((RY, q, 0, SRC_WEIGHT, l * 2 * n + q))
        for q in range(n):
            g.append((RZ, q, 0, SRC_WEIGHT, l * 2 * n + n + q))
        if entangler == "ring" and n >= 2:
            for i in range(n):
                g.append((CNOT, i, (i + 1) % n, SRC_NONE, 0))
        elif entangler == "ladder":
            for i in range(n - 1):
                g.append((CZ, i, i + 1, SRC_NONE, 0))
    gates = np.array(g, dtype=np.int32).reshape(-1, 5)
    return Circuit(n=n, gates=gates, n_inputs=n, n_weights=2 * n * layers,
                   masks=z_masks(n, extra_masks), name=name)


def paper_ansatz(n: int, depth: int, entangler: str = "chain", n_obs: int | None = None,
                 name: str = "") -> Circuit:
    """The benchmark ansatz of Sec. III-A, Eq. (7): U = U_d ... U_1 with data
    re-uploading and trainable input scaling.

    The paper fixes only the ingredients (single-qubit rotations, nearest-
    neighbour CNOTs, variational theta and scaling lambda, parameter count
    linear in n and d) and the count 168 at n=12, d=3 (Tab. I caption), i.e.
    (4d + 2) n.  The layout chosen here meets that count: block l applies
    variational RZ(theta) and RY(theta) on every qubit, the CNOT entangler
    (open chain i -> i+1, or ring), then the encoding RY(lambda s_q) and
    RZ(lambda s_q) on every qubit q; a final variational RZ, RY layer closes
    the circuit.  Weights are laid out as [theta (2n(d+1)), lambda (2nd)] so
    that the two parameter sets can take separate hyperparameters (Sec. II-C).
    Observables: Z on qubit q for the first min(n_obs, n) (default n); beyond
    n (Tab. I goes to 32 observables on 12 qubits without saying which), the
    two-qubit strings Z_i Z_(i+s) mod n for s = 1, 2, ... and i = 0..n-1.
    """
    if entangler not in ("chain", "ring"):
        raise ValueError(entangler)
    n_theta = 2 * n * (depth + 1)
    g = []

    def variational(l):
        for q in range(n):
            g.append((RZ, q, 0, SRC_WEIGHT, l * 2 * n + q))
        for q in range(n):
            g.append((RY, q, 0, SRC_WEIGHT, l * 2 * n + n + q))

    for l in range(depth):
        variational(l)
        if n >= 2:
            last = n if entangler == "ring" and n >= 3 else n - 1
            for i in range(last):
                g.append((CNOT, i, (i + 1) % n, SRC_NONE, 0))
        for q in range(n):
            g.append((RY, q, n_theta + l * 2 * n + q, SRC_SCALED, q))
        for q in range(n):
            g.append((RZ, q, n_theta + l * 2 * n + n + q, SRC_SCALED, q))
    variational(depth)
    M = n if n_obs is None else n_obs
    masks = [1 << q for q in range(min(M, n))]
    for k in range(M - n):
        i, s = k % n, 1 + k // n
        if n < 2 or s >= n:
            raise ValueError(f"{M} observables is too many for {n} qubits")
        masks.append((1 << i) | (1 << ((i + s) % n)))
    return Circuit(n=n, gates=np.array(g, dtype=np.int32).reshape(-1, 5), n_inputs=n,
                   n_weights=n_theta + 2 * n * depth, masks=np.array(masks, dtype=np.uint64),
                   name=name or f"paper_n{n}_d{depth}_{entangler}_M{M}")


def paper_workload(n: int, depth: int, batch: int, seed: int, entangler: str = "chain",
                   n_obs: int | None = None) -> Workload:
    """Seeded inputs for `paper_ansatz`: theta ~ U(-pi, pi), lambda ~ U(0.5, 1.5)
    (scalings near one), inputs s ~ U(-pi, pi), G ~ U(-1, 1), drawn in that
    order."""
    circ = paper_ansatz(n, depth, entangler, n_obs)
    rng = np.random.default_rng(seed)
    n_theta = 2 * n * (depth + 1)
    th = rng.uniform(-math.pi, math.pi, size=n_theta)
    lam = rng.uniform(0.5, 1.5, size=circ.n_weights - n_theta)
    x = rng.uniform(-math.pi, math.pi, size=(batch, circ.n_inputs))
    G = rng.uniform(-1.0, 1.0, size=(batch, circ.n_obs))
    return Workload(circuit=circ, batch=batch, inputs=x, weights=np.concatenate([th, lam]),
                    grad_out=G, meta=dict(theta=n_theta))


def _draw(rng, circ: Circuit, batch: int):
    w = rng.uniform(-math.pi, math.pi, size=circ.n_weights)
    x = rng.uniform(-math.pi, math.pi, size=(batch, circ.n_inputs))
    G = rng.uniform(-1.0, 1.0, size=(batch, circ.n_obs))
    return x, w, G


# name -> (n, layers, entangler, batch, extra masks, seed, state precision)
CONFIGS = {
    "c1": dict(n=4, layers=2, entangler="ring", batch=8, extra=(), seed=1001,
               precision="c128"),
    "c2": dict(n=12, layers=4, entangler="ring", batch=256, extra=(0xFFF,),
               seed=1002, precision="c64"),
    "c3": dict(n=20, layers=8, entangler="ladder", batch=64, extra=(),
               seed=1003, precision="c64"),
    "c5": dict(n=26, layers=10, entangler="ring", batch=16, extra=(),
               seed=1005, precision="c64"),
}

WORKLOAD_NAMES = {
    "c1": "n4_L2_ring_B8_c128",
    "c2": "n12_L4_ring_B256_c64",
    "c3": "n20_L8_czladder_B64_c64",
    "c4": "uneven1024_n8-16_L2-10_ring_c64",
    "c5": "n26_L10_ring_B16_c64",
}


def config_workload(name: str, batch: int | None = None) -> Workload:
    """Seeded inputs for a named configuration (c1, c2, c3, c5)."""
    c = CONFIGS[name]
    circ = layered_circuit(c["n"], c["layers"], c["entangler"], c["extra"],
                           name=WORKLOAD_NAMES[name])
    B = c["batch"]
    rng = np.random.default_rng(c["seed"])
    x, w, G = _draw(rng, circ, B)
    if batch is not None:
        x, G = x[:batch].copy(), G[:batch].copy()
        B = batch
    return Workload(circuit=circ, batch=B, inputs=x, weights=w, grad_out=G,
                    meta=dict(config=name, precision=c["precision"]))


def uneven_items(count: int = 1024, seed: int = 1004, n_range=(8, 16),
                 l_range=(2, 10)) -> list[Workload]:
    """Uneven batch: per item draw n, then L (inclusive ranges), then that
    item's weights, inputs (batch 1) and G."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        L = int(rng.integers(l_range[0], l_range[1] + 1))
        circ = layered_circuit(n, L, "ring", name=f"item{i}_n{n}_L{L}")
        x, w, G = _draw(rng, circ, 1)
        out.append(Workload(circuit=circ, batch=1, inputs=x, weights=w,
                            grad_out=G, meta=dict(item=i)))
    return out


def random_circuit(rng, n: int, n_gates: int, n_inputs: int = 3,
                   n_weights: int = 5, n_obs: int = 3, scaled: float = 0.0,
                   extended: float = 0.0) -> Circuit:
    """Random gate list over all gate types and random qubit pairs, with
    random parameter slots (parameters may be shared between gates).  With
    ``scaled`` > 0 that fraction of the rotations reads a weight-scaled input;
    with ``extended`` > 0 that fraction of the gates is a fixed one-qubit gate
    or (n >= 2) a controlled rotation."""
    g = []
    for _ in range(n_gates):
        if extended > 0 and rng.random() < extended:
            if n >= 2 and rng.random() < 0.4:
                t = int(rng.choice(CONTROLLED_TYPES))
                a, b = rng.choice(n, size=2, replace=False)
                if rng.random() < 0.4:
                    g.append((t, int(a), int(b), SRC_INPUT, int(rng.integers(0, n_inputs))))
                else:
                    g.append((t, int(a), int(b), SRC_WEIGHT, int(rng.integers(0, n_weights))))
            else:
                g.append((int(rng.choice(FIXED_TYPES)), int(rng.integers(0, n)), 0, SRC_NONE, 0))
            continue
        t = int(rng.integers(0, 5)) if n >= 2 else int(rng.integers(0, 3))
        if t in PARAM_TYPES:
            q = int(rng.integers(0, n))
            if scaled > 0 and rng.random() < scaled:
                g.append((t, q, int(rng.integers(0, n_weights)), SRC_SCALED,
                          int(rng.integers(0, n_inputs))))
            elif rng.random() < 0.4:
                g.append((t, q, 0, SRC_INPUT, int(rng.integers(0, n_inputs))))
            else:
                g.append((t, q, 0, SRC_WEIGHT, int(rng.integers(0, n_weights))))
        else:
            a, b = rng.choice(n, size=2, replace=False)
            g.append((t, int(a), int(b), SRC_NONE, 0))
    masks = rng.integers(1, 1 << n, size=n_obs, dtype=np.uint64)
    return Circuit(n=n, gates=np.array(g, dtype=np.int32).reshape(-1, 5),
                   n_inputs=n_inputs, n_weights=n_weights, masks=masks,
                   name=f"random_n{n}_g{n_gates}")


def random_workload(rng, circ: Circuit, batch: int) -> Workload:
    x, w, G = _draw(rng, circ, batch)
    return Workload(circuit=circ, batch=batch, inputs=x, weights=w, grad_out=G)
