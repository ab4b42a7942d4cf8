"""torch.autograd wrapper of sigma = H(h, g) v.

Forward and backward both run in libsfci (``sfci_sigma`` / ``sfci_sigma_backward``);
this module only moves arguments.  h and g are host float64 tensors (they are
uploaded to the device for each call), v is a sparse vector given as device
(rank, amplitude) tensors.  The gradients with respect to h and g are the
derivatives along symmetric perturbations.
"""
from __future__ import annotations

import torch

from . import sfci


class _SigmaFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, g, v_amp, v_rank, space, deterministic):
        n, na, nb = space
        P = sfci.Problem(n, na, nb, h.detach().cpu().numpy(), g.detach().cpu().numpy())
        r, a, _ = P.sigma(v_rank, v_amp.detach(), M=None, dedup="sort" if deterministic else "auto",
                          deterministic=deterministic)
        ctx.P = P
        ctx.h_dev, ctx.g_dev = h.device, g.device
        ctx.save_for_backward(v_rank, v_amp.detach(), r)
        ctx.mark_non_differentiable(r)
        return a, r

    @staticmethod
    def backward(ctx, grad_a, grad_r):
        v_rank, v_amp, r = ctx.saved_tensors
        vbar, dh, dg = ctx.P.sigma_backward(v_rank, v_amp, r, grad_a.contiguous())
        return dh.to(ctx.h_dev), dg.to(ctx.g_dev), vbar, None, None, None


def sigma(h, g, v_rank, v_amp, n, na, nb, deterministic=False):
    """Differentiable sigma = H v.  Returns (amplitudes, ranks) of the full (untruncated) result."""
    return _SigmaFn.apply(h, g, v_amp, v_rank, (int(n), int(na), int(nb)), bool(deterministic))
