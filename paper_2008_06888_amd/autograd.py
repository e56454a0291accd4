"""torch.autograd.Function over the library's forward and backward calls.

Forward returns E* per instance; backward returns grad_E * dE*/dJ_ij with
dE*/dJ_ij = -s_i s_j and grad_E * dE*/dh_i with dE*/dh_i = -s_i, where s is
the ground state found by the argmax-routing walk (Sec. IV: reverse-mode
differentiation of the contraction with respect to the tensor elements).
E* is piecewise linear in (J, h); at a degenerate ground state this is one
subgradient.
"""
from __future__ import annotations

import torch

from . import binding


class GroundStateEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, J, h, plan):
        if h is not None and not plan.has_field:
            raise ValueError("plan has no fields")
        energy, sigma, dJ, dh = binding.backward(plan, J.contiguous(), None if h is None else h.contiguous())
        ctx.save_for_backward(dJ, dh if dh is not None else torch.empty(0, device=J.device))
        ctx.has_h = h is not None
        ctx.sigma = sigma
        return energy

    @staticmethod
    def backward(ctx, gE):
        dJ, dh = ctx.saved_tensors
        g = gE.to(torch.float32)[:, None]
        gJ = g * dJ
        gh = (g * dh) if ctx.has_h else None
        return gJ, gh, None


def ground_state_energy(J, h, plan):
    """E* [batch] (float64), differentiable in J (and h)."""
    return GroundStateEnergy.apply(J, h, plan)
