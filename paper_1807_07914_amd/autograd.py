"""torch.autograd binding of the library's adjoint sweep.

``expectation(params, build_ops, param_index, n, hamiltonian)`` returns
E(theta) = <0| U(theta)^dag H U(theta) |0> as a 0-d float64 tensor whose
gradient with respect to ``params`` comes from qsv_adjoint.  ``build_ops(theta)``
turns a NumPy parameter vector into gate records; ``param_index[k]`` is the
parameter read by op k (-1 for ops without one).  A parameter used by several
ops receives the sum of their derivatives.

The forward pass applies the circuit (fused tile passes) and reduces E; the
output state stays on the GPU with the autograd node.  The backward pass runs
the reverse sweep from that state (lambda = H psi, then every op undone on
both vectors with each rotation's gradient term), so a forward pass costs one
circuit application whether or not a gradient is asked for, and forward plus
backward cost what one qsv_adjoint call costs.  With a caller-provided
``state``, backward must run before that state's next forward; it raises
otherwise, as it does on a second backward of the same node.
"""
from __future__ import annotations

import numpy as np
import torch

from .qsv import OpList, State


class _Expectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, build_ops, param_index, n, hamiltonian, dtype, mode, state):
        theta = params.detach().to("cpu", torch.float64).numpy()
        ol = OpList(build_ops(theta))
        s = state if state is not None else State(n, dtype)
        owned = state is None
        try:
            s.set_basis(0)
            s.apply_circuit(ol, mode=mode)
            e = s.expval(hamiltonian)
        except Exception:
            if owned:
                s.close()
            raise
        if ctx.needs_input_grad[0]:
            token = object()
            s._autograd_token = token
            ctx.qsv = (s, owned, token, ol, hamiltonian, mode,
                       np.asarray(param_index, dtype=np.int64), theta.size)
        elif owned:
            s.close()
        return torch.tensor(e, dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(ctx, grad_out):
        s, owned, token, ol, hamiltonian, mode, idx, npar = ctx.qsv
        if getattr(s, "_autograd_token", None) is not token:
            raise RuntimeError("the state no longer holds this node's forward output: run backward "
                               "before the state's next forward, and only once")
        try:
            _, g_ops = s.adjoint(ol, hamiltonian, mode=mode, state_is_output=True)
        finally:
            s._autograd_token = None
            if owned:
                s.close()
        g = np.zeros(npar, dtype=np.float64)
        sel = idx >= 0
        np.add.at(g, idx[sel], g_ops[sel])
        return (grad_out * torch.from_numpy(g).to(grad_out.device, grad_out.dtype),
                None, None, None, None, None, None, None)


def expectation(params, build_ops, param_index, n, hamiltonian, dtype="c64", mode="auto",
                state=None):
    return _Expectation.apply(params, build_ops, param_index, n, hamiltonian, dtype, mode, state)
