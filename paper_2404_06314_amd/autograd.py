"""torch.autograd integration (paper Sec. II-C): a Function whose forward is
qtm_forward and whose backward is the adjoint VJP qtm_backward, plus a small
module holding the trainable weights."""
from __future__ import annotations

import math
import warnings

import torch

from . import QTM_OPT_JIT, Circuit, precision_code


class QtmFunction(torch.autograd.Function):
    """expvals = QtmFunction.apply(inputs (B, n_in) f64, weights (n_w,) f64, circuit, precision)."""

    @staticmethod
    def forward(ctx, inputs, weights, circuit: Circuit, precision):
        inputs = inputs.contiguous()
        weights = weights.contiguous()
        prec = precision_code(precision)
        state = circuit.alloc_state(int(inputs.shape[0]), prec, device=inputs.device)
        out = circuit.forward(inputs, weights, prec, state=state)
        ctx.save_for_backward(inputs, weights)
        ctx.circuit = circuit
        ctx.precision = prec
        ctx.state = state
        return out

    @staticmethod
    def backward(ctx, grad_out):
        inputs, weights = ctx.saved_tensors
        # the saved state is un-computed by the first backward; a second
        # backward (retain_graph) recomputes the forward inside the library
        state, ctx.state = ctx.state, None
        gw, gx = ctx.circuit.backward(inputs, weights, grad_out.contiguous(), ctx.precision,
                                      state=state, need_inputs=ctx.needs_input_grad[0])
        return (gx if ctx.needs_input_grad[0] else None,
                gw if ctx.needs_input_grad[1] else None, None, None)


class QuantumLayer(torch.nn.Module):
    """Circuit with trainable weights; forward(inputs) -> (B, M) expectation values.

    Weights are initialised uniformly in [0, 2 pi) like the paper's
    ``variational_params_initial="uniform"`` (Sec. II-D) unless given.

    ``param_sets`` splits the weight vector, in slot order, into separately
    registered parameters (Sec. II-C: the variational theta and the input
    scaling lambda take their own initialisation and optimiser
    hyperparameters).  Each entry is (name, size, init) with init one of
    "uniform" (U[0, 2 pi)), "ones", "zeros", a number (constant) or a tensor
    of that size; the sizes must add up to the circuit's weight count.

    ``specialised`` runs the sweep kernels generated and compiled for this
    circuit (QTM_OPT_JIT): a one-off compile of a few seconds on the first
    call, then 2-4x faster steps from about 14 qubits on.  The default
    (None) turns them on from SPECIALISED_FROM_QUBITS qubits.

    ``drift_tol`` (a float, default None) turns on the norm-drift watchdog:
    after each forward the squared norms of the final states
    (qtm_forward_norms, 1 in exact arithmetic) are read back, which waits
    for the stream, and a RuntimeWarning is issued when one is further than
    ``drift_tol`` from 1; ``last_drift`` keeps the largest distance seen in
    the last forward.
    """

    SPECIALISED_FROM_QUBITS = 14

    def __init__(self, circuit: Circuit, precision="c64", weights=None, device="cuda",
                 param_sets=None, specialised=None, drift_tol=None):
        super().__init__()
        self.circuit = circuit
        self.precision = precision
        self.drift_tol = drift_tol
        self.last_drift = None
        if specialised is None:
            specialised = circuit.n >= self.SPECIALISED_FROM_QUBITS
        if specialised:
            circuit.set_option(QTM_OPT_JIT, 1)
        if param_sets is None:
            if weights is None:
                weights = torch.rand(circuit.n_weights, dtype=torch.float64) * (2 * math.pi)
            param_sets = [("weights", circuit.n_weights, weights)]
        elif weights is not None:
            raise ValueError("give either weights or param_sets")
        if sum(int(s) for _, s, _ in param_sets) != circuit.n_weights:
            raise ValueError("param_sets sizes must add up to the circuit's weight count")
        self._sets = []
        for name, size, init in param_sets:
            t = _initial(int(size), init).to(device)
            self.register_parameter(name, torch.nn.Parameter(t))
            self._sets.append(name)

    @classmethod
    def eq7(cls, n: int, depth: int, entangler="chain", observables=None, precision="c64",
            device="cuda", theta_init="uniform", lambda_init="ones", specialised=None):
        """The paper's benchmark ansatz (Eq. (7)) with parameter sets
        ``theta`` and ``lambda``; observables: Z masks (default Z on every
        qubit)."""
        from .ansatz import eq7_gates, z_observables
        gates, n_th, n_lam = eq7_gates(n, depth, entangler)
        masks = z_observables(n) if observables is None else observables
        circ = Circuit(n, gates, n, n_th + n_lam, masks)
        return cls(circ, precision, device=device,
                   param_sets=[("theta", n_th, theta_init), ("lambda", n_lam, lambda_init)],
                   specialised=specialised)

    @property
    def weights_vector(self):
        """All weights in slot order (a view when there is one set)."""
        ps = [getattr(self, n) for n in self._sets]
        return ps[0] if len(ps) == 1 else torch.cat(ps)

    def param_groups(self, **hyper):
        """Optimiser groups, one per parameter set: ``param_groups(theta=dict(lr=0.01),
        lambda_=dict(lr=0.1))`` (a trailing underscore may be used for names that
        are Python keywords)."""
        groups = []
        for n in self._sets:
            h = hyper.get(n, hyper.get(n + "_", {}))
            groups.append(dict(params=[getattr(self, n)], **h))
        return groups

    def forward(self, inputs):
        out = QtmFunction.apply(inputs.to(torch.float64), self.weights_vector, self.circuit,
                                self.precision)
        if self.drift_tol is not None:
            nr = self.circuit.forward_norms(int(inputs.shape[0]))
            self.last_drift = float(torch.max(torch.abs(nr - 1.0)).item())
            if self.last_drift > self.drift_tol:
                warnings.warn(f"state norm drifted by {self.last_drift:.3e} (> {self.drift_tol:g}) "
                              "in the last forward", RuntimeWarning)
        return out


def _initial(size: int, init):
    if isinstance(init, str):
        if init == "uniform":
            return torch.rand(size, dtype=torch.float64) * (2 * math.pi)
        if init == "ones":
            return torch.ones(size, dtype=torch.float64)
        if init == "zeros":
            return torch.zeros(size, dtype=torch.float64)
        raise ValueError(f"unknown init {init!r}")
    if isinstance(init, (int, float)):
        return torch.full((size,), float(init), dtype=torch.float64)
    t = torch.as_tensor(init, dtype=torch.float64).reshape(-1).clone()
    if t.numel() != size:
        raise ValueError(f"initial values have {t.numel()} entries, expected {size}")
    return t


# The paper's module name for a circuit with trainable weights (Sec. II-D).
QuantumModule = QuantumLayer


class HybridModule(torch.nn.Module):
    """End-to-end differentiable hybrid model (Sec. II-C): a classical fully
    connected pre-processing layer (input_size -> n_qubits) whose outputs are
    the data s encoded in the circuit, the Eq. (7) quantum layer with Z on
    every qubit (parameter sets theta and lambda), and a classical fully
    connected post-processing layer (n_qubits -> output_size).  The gradient
    reaches the pre-processing layer through dL/dinputs of the adjoint pass.
    """

    def __init__(self, input_size: int, output_size: int, n_qubits: int, depth: int,
                 entangler="chain", precision="c64", device="cuda", theta_init="uniform",
                 lambda_init="ones", specialised=None):
        super().__init__()
        self.pre = torch.nn.Linear(input_size, n_qubits, dtype=torch.float64, device=device)
        self.quantum = QuantumLayer.eq7(n_qubits, depth, entangler=entangler, precision=precision,
                                        device=device, theta_init=theta_init,
                                        lambda_init=lambda_init, specialised=specialised)
        self.post = torch.nn.Linear(n_qubits, output_size, dtype=torch.float64, device=device)

    def forward(self, x):
        return self.post(self.quantum(self.pre(x.to(torch.float64))))
