"""Effective stiffness as a differentiable torch function of the voxel moduli.

forward:  C* = cell_effective_stiffness(E, nu)            (HIP library)
backward: dL/dE = cell_adjoint(dL/dC*)                     (HIP library)

The cell problem is self-adjoint and C* is a stationary value of the
energy, so the adjoint states are the primal solutions of the forward call
and the backward pass is a single per-voxel kernel (no extra solve).  Torch
only supplies tensors; the solve and the gradient run in the library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding


class EffectiveStiffness(torch.autograd.Function):
    """C* (nv x nv, float64) from per-voxel E (float64, n values).

    ``cell`` is a ``binding.Cell`` of matching shape; it must not run another
    solve between this forward and its backward (checked).  ``nu`` is a
    constant (no gradient).
    """

    @staticmethod
    def forward(ctx, E, nu, cell):
        if E.dtype != torch.float64:
            raise TypeError("E must be float64")
        cell.set_material(E.detach().contiguous(), nu.detach().to(E.device).contiguous())
        C, info = cell.effective_stiffness()
        ctx.cell = cell
        ctx.solve_id = cell.solves
        ctx.device = E.device
        ctx.info = info
        return torch.from_numpy(C).to(E.device)

    @staticmethod
    def backward(ctx, grad_C):
        cell = ctx.cell
        if cell.solves != ctx.solve_id:
            raise RuntimeError("the cell ran another solve between forward and backward")
        a = grad_C.detach().to("cpu", torch.float64).numpy()
        if ctx.device.type == "cuda":
            g = torch.empty(cell.n, dtype=torch.float64, device=ctx.device)
            cell.adjoint(a, out=g)
        else:
            g = torch.from_numpy(cell.adjoint(a))
        return g, None, None


def effective_stiffness(E, nu, cell):
    """Differentiable C*(E) on an existing cell handle."""
    return EffectiveStiffness.apply(E, nu, cell)
