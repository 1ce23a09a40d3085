"""Reference detectors of the paper's comparison (test infrastructure only).

Section V-A compares TASER with linear MMSE detection, the K-best algorithm
(K = 5) and ML detection; the matched filter is TASER's own one-iteration
limit.  These are plain float64 numpy restatements on the real-valued model
of Section II-A (ybar = Hbar sbar + nbar with sbar in {-1, +1}^(N-1)), with a
library linear solve or QR factorisation as single steps.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
this module; it shares no code with the HIP path.

Readings where the paper gives only a citation:
  * MMSE uses the real-valued model with unit symbol energy per real
    dimension and noise variance N0/2 per real dimension:
    xhat = (Hbar^T Hbar + (N0/2) I)^-1 Hbar^T ybar (for QPSK this is the
    complex MMSE (H^H H + (N0/Es) I)^-1 H^H y with Es = 2);
  * K-best runs breadth first on the real-valued model after a QR
    factorisation Hbar = Q R (R upper triangular, positive diagonal): from
    the last real dimension to the first, every surviving path is extended
    by both values +-1 and the K paths of smallest partial distance
    sum_l (z_l - sum_m R_lm s_m)^2, z = Q^T ybar, survive (ties: the earlier
    candidate in the order path rank, then +1 before -1);
  * decisions are signs with sign(0) = +1, in the order s~ of Section II-A.
"""
from __future__ import annotations

import numpy as np

from .taser import real_decomposition_coherent


def _sign(x):
    return np.where(np.asarray(x) >= 0.0, 1, -1).astype(np.int8)


def matched_filter(H, y, mod):
    """xhat = Hbar^T ybar (the matched filter; Algorithm 1 after one
    iteration has the same signs).  Returns (sbar, xhat)."""
    Hbar, ybar = real_decomposition_coherent(H, y, mod)
    x = np.einsum("...bu,...b->...u", Hbar, ybar)
    return _sign(x), x


def mmse(H, y, mod, n0):
    """Linear MMSE on the real-valued model: (Hbar^T Hbar + (N0/2) I) xhat =
    Hbar^T ybar.  n0: the complex noise variance N0 (scalar or [...]).
    Returns (sbar, xhat)."""
    Hbar, ybar = real_decomposition_coherent(H, y, mod)
    G = np.swapaxes(Hbar, -1, -2) @ Hbar
    M = G.shape[-1]
    reg = (np.asarray(n0, dtype=np.float64) / 2.0)[..., None, None] * np.eye(M)
    b = np.einsum("...bu,...b->...u", Hbar, ybar)
    x = np.linalg.solve(G + reg, b[..., None])[..., 0]
    return _sign(x), x


def kbest(H, y, mod, K, return_gap=False):
    """K-best breadth-first tree search (see the module docstring).
    H [V, B, U], y [V, B].  Returns (sbar [V, N-1], metric [V]) with metric
    the partial distance ||z - R shat||^2 of the surviving best path; with
    return_gap also the smallest relative gap, over the levels where paths
    were dropped, between the K-th kept and the best dropped partial
    distance (a near-tie there lets rounding change the survivors)."""
    Hbar, ybar = real_decomposition_coherent(H, y, mod)
    V, _, M = Hbar.shape
    sbar = np.zeros((V, M), dtype=np.int8)
    metric = np.zeros(V)
    gap = np.full(V, np.inf)
    for v in range(V):
        Q, R = np.linalg.qr(Hbar[v])                  # reduced: Q [2B, M], R [M, M]
        d = np.sign(np.diag(R))
        d[d == 0] = 1.0
        R = d[:, None] * R                            # positive diagonal
        z = d * (Q.T @ ybar[v])
        paths = [((), 0.0)]                           # (s_i..s_{M-1}, partial distance)
        for i in range(M - 1, -1, -1):
            cand = []
            for rank, (s, pd) in enumerate(paths):
                tail = np.array(s, dtype=np.float64)
                above = R[i, i + 1:] @ tail if len(s) else 0.0
                for sym in (1.0, -1.0):
                    e = z[i] - R[i, i] * sym - above
                    cand.append((pd + e * e, rank, -sym, (sym,) + s))
            cand.sort(key=lambda c: (c[0], c[1], c[2]))
            if len(cand) > K:
                hi = cand[K][0]
                gap[v] = min(gap[v], (hi - cand[K - 1][0]) / max(hi, 1e-300))
            paths = [(c[3], c[0]) for c in cand[:K]]
        best = paths[0]
        sbar[v] = np.array(best[0], dtype=np.int8)
        metric[v] = best[1]
    if return_gap:
        return sbar, metric, gap
    return sbar, metric


def residual(H, y, mod, sbar):
    """||ybar - Hbar sbar||^2 of given decisions (the ML objective of
    eq. (1)), float64."""
    Hbar, ybar = real_decomposition_coherent(H, y, mod)
    r = ybar - np.einsum("...bu,...u->...b", Hbar, np.asarray(sbar, dtype=np.float64))
    return np.sum(r * r, axis=-1)
