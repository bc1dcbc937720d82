"""dF/dJ through torch autograd: the regularized OTOC F(t*) of the Chebyshev
forward as a differentiable function of the couplings J.  The library's
reverse sweep (syk_grad_couplings) supplies the gradient; nothing here
differentiates numerically."""
from __future__ import annotations

import numpy as np
import torch

from . import api


class ChebOTOC(torch.autograd.Function):
    """F = ChebOTOC.apply(J, N, i, j, beta, t_star, psi0, opts).

    J: float64 CPU tensor of C(N,4) couplings (lexicographic quartets).
    psi0: complex128 GPU state of dimension 2^(N/2).  opts: api.cheb_opts(...).
    Returns a 0-dim float64 CPU tensor."""

    @staticmethod
    def forward(ctx, J, N, i, j, beta, t_star, psi0, opts):
        if J.dtype != torch.float64 or J.device.type != "cpu":
            raise TypeError("J must be a float64 CPU tensor")
        T = api.Terms(N, J.detach().numpy())
        try:
            if ctx.needs_input_grad[0]:
                F, g = api.grad_couplings(T, i, j, beta, t_star, psi0, opts)
                ctx.save_for_backward(torch.from_numpy(g))
            else:
                F = api.cheb_otoc(T, i, j, beta, t_star, psi0, opts)
        finally:
            T.close()
        return torch.tensor(F, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gF):
        (g,) = ctx.saved_tensors
        return (gF * g, None, None, None, None, None, None, None)


def otoc_value_and_grad(J: np.ndarray, N: int, i: int, j: int, beta: float, t_star: float, psi0, opts):
    """Convenience: (F, dF/dJ) as numpy via autograd."""
    Jt = torch.from_numpy(np.ascontiguousarray(J, dtype=np.float64)).requires_grad_(True)
    F = ChebOTOC.apply(Jt, N, i, j, beta, t_star, psi0, opts)
    F.backward()
    return float(F.detach()), Jt.grad.numpy().copy()
