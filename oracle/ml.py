"""Exhaustive maximum-likelihood detectors (test infrastructure only).

They enumerate every candidate and evaluate the paper's objectives in complex
arithmetic, with no real-valued reformulation, so they pin the oracle's T
construction from outside.  Sizes are tiny: at most 2^12 candidates.
"""
from __future__ import annotations

import itertools

import numpy as np

BPSK = 1
QPSK = 2


def constellation(mod):
    if mod == QPSK:
        return np.array([1 + 1j, 1 - 1j, -1 + 1j, -1 - 1j])
    return np.array([1.0 + 0j, -1.0 + 0j])


def candidates(count, mod):
    """All vectors in O^count, shape [|O|^count, count]."""
    pts = constellation(mod)
    return np.array(list(itertools.product(pts, repeat=count)), dtype=np.complex128)


def ml_coherent(H, y, mod):
    """eq. (1): argmin_{s in O^U} ||y - H s||_2.  H [..., B, U], y [..., B].
    Returns (s_ml [..., U], cost [...] = ||y - H s_ml||^2)."""
    H = np.asarray(H).astype(np.complex128)
    y = np.asarray(y).astype(np.complex128)
    U = H.shape[-1]
    S = candidates(U, mod)                                # [C, U]
    r = y[..., None, :] - np.einsum("...bu,cu->...cb", H, S)
    cost = np.sum(np.abs(r) ** 2, axis=-1)                # [..., C]
    idx = np.argmin(cost, axis=-1)
    return S[idx], np.take_along_axis(cost, idx[..., None], axis=-1)[..., 0]


def ml_jed(Y, s0, mod):
    """eq. (3)/(4) with a known first symbol: argmax_{s_r} ||y0 s0 + Y_r s_r||.
    Y [..., K+1, B] slot-major.  Returns (s_r [..., K], value [...] = the
    maximal ||Y s||^2)."""
    Y = np.asarray(Y).astype(np.complex128)
    s0 = np.asarray(s0).astype(np.complex128)
    K = Y.shape[-2] - 1
    S = candidates(K, mod)                                # [C, K]
    base = Y[..., 0, :] * s0[..., None]                   # [..., B]
    z = base[..., None, :] + np.einsum("...kb,ck->...cb", Y[..., 1:, :], S)
    val = np.sum(np.abs(z) ** 2, axis=-1)
    idx = np.argmax(val, axis=-1)
    return S[idx], np.take_along_axis(val, idx[..., None], axis=-1)[..., 0]


def ml_over_T(T):
    """argmin over s~ = [sbar; 1] with sbar in {-1,+1}^(N-1) of s~^T T s~
    (eq. (2) / eq. (5) as written).  T [..., N, N].  Returns (sbar, value)."""
    T = np.asarray(T, dtype=np.float64)
    N = T.shape[-1]
    S = np.array(list(itertools.product([1.0, -1.0], repeat=N - 1)))
    St = np.concatenate([S, np.ones((S.shape[0], 1))], axis=1)      # [C, N]
    val = np.einsum("cn,...nm,cm->...c", St, T, St)
    idx = np.argmin(val, axis=-1)
    return S[idx].astype(np.int8), np.take_along_axis(val, idx[..., None], axis=-1)[..., 0]
