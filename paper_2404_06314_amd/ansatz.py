"""Gate lists for the paper's benchmark ansatz (Sec. III-A, Eq. (7)).

U = U_d ... U_1, each block with variational single-qubit rotations, a
nearest-neighbour CNOT entangler and data re-uploading with trainable input
scaling (angle lambda * s).  The paper fixes the ingredients and the count
of (4d + 2) n trainable parameters (168 at n = 12, d = 3, Tab. I caption);
the order within a block is a choice: RZ(theta), RY(theta) on every qubit,
the CNOTs (open chain i -> i+1, or ring with the wrap gate last), then
RY(lambda s_q), RZ(lambda s_q) on every qubit; a final RZ, RY layer of
theta closes the circuit.  Weight slots: theta first (2n(d+1), construction
order), then lambda (2nd), so the two sets are contiguous.
"""
from __future__ import annotations

import numpy as np

from ._lib import QTM_CNOT, QTM_RY, QTM_RZ, QTM_SRC_NONE, QTM_SRC_SCALED, QTM_SRC_WEIGHT


def eq7_gates(n: int, depth: int, entangler: str = "chain"):
    """Returns (gates int32 [G, 5], n_theta, n_lambda)."""
    if n < 1 or depth < 0:
        raise ValueError("need n >= 1 and depth >= 0")
    if entangler not in ("chain", "ring"):
        raise ValueError(f"unknown entangler {entangler!r}")
    n_theta = 2 * n * (depth + 1)
    g = []

    def variational(l):
        g.extend((QTM_RZ, q, 0, QTM_SRC_WEIGHT, 2 * n * l + q) for q in range(n))
        g.extend((QTM_RY, q, 0, QTM_SRC_WEIGHT, 2 * n * l + n + q) for q in range(n))

    for l in range(depth):
        variational(l)
        if n >= 2:
            m = n if (entangler == "ring" and n >= 3) else n - 1
            g.extend((QTM_CNOT, i, (i + 1) % n, QTM_SRC_NONE, 0) for i in range(m))
        base = n_theta + 2 * n * l
        g.extend((QTM_RY, q, base + q, QTM_SRC_SCALED, q) for q in range(n))
        g.extend((QTM_RZ, q, base + n + q, QTM_SRC_SCALED, q) for q in range(n))
    variational(depth)
    return np.array(g, dtype=np.int32).reshape(-1, 5), n_theta, 2 * n * depth


def z_observables(n: int, qubits=None) -> np.ndarray:
    """Single-qubit Z masks (default: every qubit, as in the paper's benchmarks)."""
    qs = range(n) if qubits is None else qubits
    return np.array([1 << int(q) for q in qs], dtype=np.uint64)
