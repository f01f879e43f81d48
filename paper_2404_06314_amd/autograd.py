"""torch.autograd integration (paper Sec. II-C): a Function whose forward is
qtm_forward and whose backward is the adjoint VJP qtm_backward, plus a small
module holding the trainable weights."""
from __future__ import annotations

import math

import torch

from . import Circuit, precision_code


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
    """

    def __init__(self, circuit: Circuit, precision="c64", weights=None, device="cuda"):
        super().__init__()
        self.circuit = circuit
        self.precision = precision
        if weights is None:
            weights = torch.rand(circuit.n_weights, dtype=torch.float64) * (2 * math.pi)
        self.weights = torch.nn.Parameter(torch.as_tensor(weights, dtype=torch.float64).to(device))

    def forward(self, inputs):
        return QtmFunction.apply(inputs.to(torch.float64), self.weights, self.circuit,
                                 self.precision)
