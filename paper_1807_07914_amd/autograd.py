"""torch.autograd binding of the library's adjoint sweep.

``expectation(params, build_ops, param_index, n, hamiltonian)`` returns
E(theta) = <0| U(theta)^dag H U(theta) |0> as a 0-d float64 tensor whose
gradient with respect to ``params`` comes from qsv_adjoint (one forward pass
and one reverse sweep on the GPU).  ``build_ops(theta)`` turns a NumPy
parameter vector into gate records; ``param_index[k]`` is the parameter read
by op k (-1 for ops without one).  A parameter used by several ops receives
the sum of their derivatives.
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
        try:
            s.set_basis(0)
            if ctx.needs_input_grad[0]:
                e, g_ops = s.adjoint(ol, hamiltonian, mode=mode)
                idx = np.asarray(param_index, dtype=np.int64)
                g = np.zeros(theta.size, dtype=np.float64)
                sel = idx >= 0
                np.add.at(g, idx[sel], g_ops[sel])
                ctx.save_for_backward(torch.from_numpy(g))
            else:
                s.apply_circuit(ol, mode=mode)
                e = s.expval(hamiltonian)
        finally:
            if state is None:
                s.close()
        return torch.tensor(e, dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return (grad_out * g.to(grad_out.device, grad_out.dtype),
                None, None, None, None, None, None, None)


def expectation(params, build_ops, param_index, n, hamiltonian, dtype="c64", mode="auto",
                state=None):
    return _Expectation.apply(params, build_ops, param_index, n, hamiltonian, dtype, mode, state)
