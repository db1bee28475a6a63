"""torch.autograd.Function over the HIP library: energy of a velocity field.

forward(v) runs the forward sweep of the semi-Lagrangian flow and returns the
energy E(v) (Methods, Registration: E = int ||L v||^2 + sigma^-2 ||J0 o phi_10 - J1||^2)
as a float64 scalar.  Nothing but v is saved: backward recomputes the maps phi_t
and runs the exact reverse sweep (adjoint of trilinear sampling by a
deterministic gather, coordinate gradient of the sampler, periodic stencils for
the regulariser), so memory does not grow with T x grid for the autograd graph.
With Params.flags = FLAG_RECOMPUTE_PHI the library itself keeps only every
`checkpoint_every`-th map during the reverse sweep and recomputes the rest.
"""

from __future__ import annotations

import torch

from . import lddmm as L


class LddmmEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, M0, M1, MI0, MI1, params, spacing, ws):
        out = L.lddmm_energy(M0, M1, MI0, MI1, v.detach().contiguous(), params, spacing, ws=ws)
        ctx.save_for_backward(v)
        ctx.extra = (M0, M1, MI0, MI1, params, spacing, ws)
        return out[0].clone()

    @staticmethod
    def backward(ctx, gE):
        (v,) = ctx.saved_tensors
        M0, M1, MI0, MI1, params, spacing, ws = ctx.extra
        grad, _ = L.lddmm_gradient(M0, M1, MI0, MI1, v.detach().contiguous(), params,
                                   kind=L.GRAD_L2, spacing=spacing, ws=ws)
        return (gE.to(grad.dtype) * grad, None, None, None, None, None, None, None)


def lddmm_energy_fn(v, M0, M1, MI0=None, MI1=None, params=None, spacing=1.0, ws=None):
    """Differentiable E(v): a float64 0-d tensor whose backward is the exact dE/dv."""
    params = params or L.Params()
    if ws is None:
        ws = L.workspace(M0.shape, params, spacing, M0.device)
    return LddmmEnergy.apply(v, M0, M1, MI0, MI1, params, spacing, ws)
