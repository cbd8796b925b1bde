"""Differentiable solvation energy.

``SolvationEnergy.apply(q, pos, tree, ...)`` returns dG(q, pos) = kappa q^T C
A^-1 f B q (kcal/mol) from the FMM-BEM solve; its backward runs the library's
hand-written adjoint (``bemfmm_adjoint_grad``: one transposed solve A^T y =
C^T q with a dipole-source FMM, then one FMM for the charge potentials and
fields) instead of differentiating through the solver.  Only the tree handle,
the charge values and positions and the forward solution x are kept between
forward and backward; every expansion is recomputed (rematerialised) in
backward, after the charges are moved back to the positions of this forward
(another forward on the same tree may have moved them since).

The triangulated surface is held fixed; ``pos`` moves the charges inside
their leaf cells of the existing tree (``bemfmm_set_charges``).
"""
from __future__ import annotations

import torch

from . import FP32_REFINED, adjoint_grad, set_charges, solvation_energy, solve_bem


class SolvationEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, pos, tree, tol=1e-8, maxit=300, restart=30, precision=FP32_REFINED):
        q = q.detach().to(torch.float64).contiguous()
        pos = pos.detach().to(torch.float64).contiguous()
        set_charges(tree, pos)
        x, info = solve_bem(tree, q, tol=tol, maxit=maxit, restart=restart, precision=precision)
        dG = solvation_energy(tree, q, x, precision=precision)
        ctx.save_for_backward(q, pos, x)
        ctx.tree = tree
        ctx.opts = (tol, maxit, restart, precision)
        ctx.forward_info = info
        return torch.tensor(dG, dtype=torch.float64, device=q.device)

    @staticmethod
    def backward(ctx, g):
        q, pos, x = ctx.saved_tensors
        tol, maxit, restart, precision = ctx.opts
        set_charges(ctx.tree, pos)
        want_q, want_pos = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dq, dpos, _ = adjoint_grad(ctx.tree, q, x, tol=tol, maxit=maxit, restart=restart, precision=precision,
                                   want_dq=want_q, want_dpos=want_pos)
        gq = g * dq if want_q else None
        gp = g * dpos if want_pos else None
        return gq, gp, None, None, None, None, None


def solvation_energy_autograd(q, pos, tree, **kw):
    """dG with gradients w.r.t. the charge values and positions."""
    return SolvationEnergy.apply(q, pos, tree, kw.get("tol", 1e-8), kw.get("maxit", 300), kw.get("restart", 30),
                                 kw.get("precision", FP32_REFINED))
