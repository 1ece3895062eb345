"""LJForce: the force map as a torch.autograd.Function.

forward runs ljmd_lj_forces (FP64 gather) and backward runs the hand-written
adjoint kernel ljmd_lj_backward, giving gradients of any scalar loss of the
forces with respect to positions and the eps/sigma tables.  Cutoffs are held
fixed; the list must be current for x.  pair_table builds the symmetric
tables from the unique type-pair parameters, so that their gradients come
out directly (an off-diagonal parameter collects both mirrored entries).
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


class LJForce(torch.autograd.Function):
    """F = LJForce.apply(x, eps, sigma, system) with system = (types, box, rc, skin,
    nl, ws).  eps and sigma are ntypes x ntypes float64 tensors (any device);
    their values enter the host-side parameter struct."""

    @staticmethod
    def forward(ctx, x, eps, sigma, system):
        types, box, rc, skin, nl, ws = system
        params = api.LJParams(eps=eps.detach().cpu().numpy(), sigma=sigma.detach().cpu().numpy(),
                              rc=np.asarray(rc), skin=skin)
        f, _ = api.lj_forces(x.detach(), types, box, params, nl, ws=ws)
        ctx.save_for_backward(x)
        ctx.params = params
        ctx.system = system
        ctx.param_device = eps.device
        return f

    @staticmethod
    def backward(ctx, gF):
        (x,) = ctx.saved_tensors
        types, box, rc, skin, nl, ws = ctx.system
        gx, geps, gsig = api.lj_backward(x.detach(), types, box, ctx.params, nl,
                                         gF.contiguous(), ws=ws)
        return gx, geps.to(ctx.param_device), gsig.to(ctx.param_device), None


def pair_table(upper: torch.Tensor, ntypes: int) -> torch.Tensor:
    """Symmetric ntypes x ntypes table from its ntypes (ntypes + 1) / 2
    unique values, row by row over the upper triangle: (0,0), (0,1), ...,
    (0,T-1), (1,1), ...  Differentiable: the gradient of an off-diagonal value
    is the sum of the gradients of its two mirrored entries."""
    if upper.shape != (ntypes * (ntypes + 1) // 2,):
        raise ValueError("upper must hold ntypes (ntypes + 1) / 2 values")
    ia, ib = torch.triu_indices(ntypes, ntypes, device=upper.device)
    table = upper.new_zeros((ntypes, ntypes))
    table = table.index_put((ia, ib), upper)
    return table.index_put((ib, ia), upper)
