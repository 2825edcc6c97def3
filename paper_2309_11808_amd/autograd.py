"""Differentiable SPOD: a torch.autograd.Function over the libspod path.

    lam, phi = spod(q, plan, n_modes=5, bins=None, keep_qhat=False)

The forward runs spod_blocks_fft, spod_csd, spod_eig and spod_modes; the
backward runs spod_backward, which recomputes the Fourier blocks (at the
selected bins only) unless keep_qhat=True kept them from the forward.  A block
length other than a power of two up to 1024 always keeps them (its transform
has no bin selection to recompute from).  With
`bins`, lam and phi are returned for those frequencies only ([nb, L] and
[nb, n_modes, M]), and the backward touches only those frequencies.

Gradients of complex outputs use PyTorch's convention, which is the one
spod_backward expects, so grad_output is passed through unchanged.
"""
from __future__ import annotations

import numpy as np
import torch

from .spod import Plan

__all__ = ["spod", "SpodFunction"]


class SpodFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, plan: Plan, n_modes: int, bins, keep_qhat: bool):
        out = plan.forward(q, n_modes)
        lam, phi = out["lam"], out["phi"]
        ctx.plan, ctx.n_modes, ctx.bins = plan, n_modes, bins
        ctx.set_materialize_grads(False)
        nf = plan.nfft
        general = not (nf & (nf - 1) == 0 and nf <= 1024)
        keep = (keep_qhat or general) and not plan.packed
        ctx.save_for_backward(q, lam, out["psi"], out["qhat"] if keep else None)
        if bins is not None:
            idx = torch.as_tensor(np.asarray(bins, dtype=np.int64), device=q.device)
            return lam.index_select(0, idx), phi.index_select(0, idx)
        return lam, phi

    @staticmethod
    def backward(ctx, g_lam, g_phi):
        q, lam, psi, qhat = ctx.saved_tensors
        if g_lam is None and g_phi is None:
            return None, None, None, None, None
        g_q = ctx.plan.backward(
            q, lam, psi,
            g_lam=None if g_lam is None else g_lam.contiguous(),
            g_phi=None if g_phi is None else g_phi.contiguous(),
            n_modes=ctx.n_modes, bins=ctx.bins, qhat=qhat)
        return g_q, None, None, None, None


def spod(q: torch.Tensor, plan: Plan, n_modes: int = 5, bins=None, keep_qhat: bool = False):
    """(lam, phi) of the SPOD of q, differentiable with respect to q."""
    if bins is not None:
        bins = [int(b) for b in bins]
    return SpodFunction.apply(q, plan, n_modes, bins, keep_qhat)
