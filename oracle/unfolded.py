"""Unfolded TASER with one step size per iteration, in plain PyTorch FP64
on the CPU (test infrastructure only).

The forward is Algorithm 1 with tau_t = alpha_t / ||T~||_2 in iteration t
(a learnable step-size schedule; with alpha_t constant it is the paper's
algorithm).  Autograd through these ordinary torch operations is the
independent reference for the hand-written adjoint.  The loss is the mean
squared error between the last row of L = L~ D^-1 and the transmitted
sbar, over the N-1 detected entries.
"""
from __future__ import annotations

import torch


def unfolded_forward(Tt, D, lam, alpha_t, pin_last=True):
    """Tt [V, N, N], D [V, N], lam [V] (= ||T~||_2), alpha_t [t_max]
    (all float64 CPU tensors).  Returns L~ after t_max iterations."""
    V, N, _ = Tt.shape
    L = torch.diag_embed(D)
    mask = torch.tril(torch.ones(N, N, dtype=Tt.dtype))
    for t in range(alpha_t.shape[0]):
        tau = (alpha_t[t] / lam)[:, None, None]
        Vm = L - mask * (2.0 * tau * (L @ Tt))
        norms = torch.sqrt(torch.sum(Vm * Vm, dim=-2))
        L = Vm * (D / norms)[:, None, :]
        if pin_last:
            last = torch.zeros(N, N, dtype=Tt.dtype)
            last[N - 1, N - 1] = 1.0
            L = L * (1.0 - last) + last * D[:, N - 1, None, None]
    return L


def last_row_mse(L, D, sbar):
    """mean_{v,k<N} (L~_{N,k}/D_kk - sbar_k)^2."""
    est = L[:, -1, :-1] / D[:, :-1]
    return torch.mean((est - sbar) ** 2)
