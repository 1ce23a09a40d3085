"""Unfolded TASER with learned per-iteration step sizes (deep unfolding of
Algorithm 1: iteration t uses tau_t = alpha_t / ||T~||_2).

``UnfoldedTaser`` is a ``torch.autograd.Function`` whose forward and backward
are the HIP kernels behind ``taser_unfolded_forward`` / ``_backward``; only
the step sizes alpha receive a gradient (T~, D and ||T~||_2 are the fixed
preprocessing of each received vector).  ``last_row`` and ``mse_loss`` give
the training objective on the detector's soft output L~_{N,k} / D_kk.
"""
from __future__ import annotations

import torch

from . import unfolded_backward, unfolded_forward


class UnfoldedTaser(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, Tt, D, lam, ckpt_every=None, literal_last=False):
        alpha = alpha.detach().contiguous()
        L, ckpt, u = unfolded_forward(Tt, D, lam, alpha, ckpt_every, literal_last)
        ctx.save_for_backward(alpha, Tt, D, lam, ckpt)
        ctx.u = u
        return L

    @staticmethod
    def backward(ctx, dL):
        alpha, Tt, D, lam, ckpt = ctx.saved_tensors
        dalpha = unfolded_backward(ctx.u, Tt, D, lam, alpha, ckpt, dL.contiguous())
        return dalpha, None, None, None, None, None


def unfolded(alpha, Tt, D, lam, ckpt_every=None, literal_last=False):
    """Packed L~ [V, N(N+1)/2] after len(alpha) iterations."""
    return UnfoldedTaser.apply(alpha, Tt, D, lam, ckpt_every, literal_last)


def last_row(L, N):
    """Row N of the packed lower triangle, entries k < N: [V, N-1]."""
    base = (N - 1) * N // 2
    return L[:, base:base + N - 1]


def soft_output(L, D):
    N = D.shape[1]
    return last_row(L, N) / D[:, :N - 1]


def mse_loss(L, D, sbar):
    """mean_{v,k} (L~_{N,k} / D_kk - sbar_k)^2, sbar in {-1, +1}."""
    return torch.mean((soft_output(L, D) - sbar) ** 2)
