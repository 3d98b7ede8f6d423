"""torch.autograd wrapper: eigenvalues forward through ``chase_ph_solve``,
backward through the library's adjoint kernel (``chase_ph_eigval_backward``).

Gradients follow PyTorch's convention for complex inputs
(``grad = dL/dRe + i dL/dIm``) and are projected on the structure the solver
assumes: Hermitian for A, complex symmetric for B.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from .solver import PHSolver


class EigvalsPH(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, W0, Lz, nev, nex, kwargs):
        solver = PHSolver(A.detach(), B.detach(), nev, nex, **kwargs)
        ev, V, res, info = solver.solve(W0, Lz)
        ctx.solver = solver
        ctx.save_for_backward(V)
        ctx.info = info
        return torch.as_tensor(ev, dtype=torch.float64, device=A.device)

    @staticmethod
    def backward(ctx, g):
        (V,) = ctx.saved_tensors
        GA, GB = ctx.solver.eigval_backward(V, g.detach().double().cpu().numpy())
        # the library writes column-major m x m; as a (m, m) tensor view this is G itself
        return GA.contiguous(), GB.contiguous(), None, None, None, None, None


def eigsh_ph(A, B, nev, nex, W0, Lz, **kwargs):
    """Smallest positive eigenvalues of H (differentiable w.r.t. A and B)."""
    return EigvalsPH.apply(A, B, W0, Lz, nev, nex, kwargs)
