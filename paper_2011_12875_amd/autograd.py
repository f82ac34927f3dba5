"""Differentiable SNAP energy: torch.autograd.Function over the C ABI.

Forward runs compute_U and the bispectrum (snap_forward) and returns the
per-atom energies E_i = sum_l beta_l B_il (eq. (snapatomenergy)).  Backward is
the adjoint of Sec. IV -- the paper notes that its Y is reverse-mode
differentiation of B with respect to U: with upstream g_i = dL/dE_i it builds
Y from the per-atom coefficients g_i * beta (compute_Y), runs the fused
derivative kernel (compute_dE) and gathers forces, so
    dL/dr     = -F(g),
    dL/dbeta  = sum_i g_i B_i   (or g_i B_i for per-atom coefficients),
the latter by the library's fixed-order reduction (snap_beta_grad).  Double
backward is not supported: the backward is once-differentiable, so asking for
a second derivative raises instead of returning a gradient without a graph.
"""
from __future__ import annotations

import torch

from . import snapmi


class _SnapEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, beta, pot, box, nl):
        pos_c = pos.detach().contiguous()
        beta_c = beta.detach().contiguous()
        E, B = pot.forward(pos_c, box, nl, beta_c)
        ctx.pot, ctx.box, ctx.nl = pot, box, nl
        ctx.token = pot._fwd_token
        ctx.save_for_backward(pos_c, beta_c, B)
        return E

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gE):
        pos, beta, B = ctx.saved_tensors
        pot = ctx.pot
        gE = gE.detach().contiguous().to(torch.float64)
        grad_pos = grad_beta = None
        if ctx.needs_input_grad[0]:
            if pot._fwd_token != ctx.token:
                # another evaluation reused the context's U since this forward
                pot.forward(pos, ctx.box, ctx.nl, beta)
            F = pot.backward(pos, ctx.box, ctx.nl, beta, gE)
            grad_pos = -F
        if ctx.needs_input_grad[1]:
            grad_beta = pot.beta_grad(gE, B, per_atom=beta.dim() == 2)
        return grad_pos, grad_beta, None, None, None


def snap_energy(pos, beta, pot: "snapmi.SnapPotential", box, nl: "snapmi.NeighborList"):
    """Per-atom SNAP energies E_i (FP64), differentiable in pos and beta."""
    return _SnapEnergy.apply(pos, beta, pot, box, nl)
