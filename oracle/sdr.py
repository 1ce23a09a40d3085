"""Exact semidefinite relaxation (SDR) detector in float64 numpy (test
infrastructure only).

eq. (7): S^ = argmin Tr(T S) subject to diag(S) = 1 and S positive
semidefinite, then (Section II-C) the estimate is read from the signs of the
leading eigenvector of S^ (exact when S^ has rank one).  T is the matrix of
eq. (2) or eq. (5).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use this module; it shares no code with
the HIP path.

The SDP is solved by a primal-dual interior-point method with the HKM
search direction, the standard method for this max-cut-type program
(Helmberg, Rendl, Vanderbei and Wolkowicz, 1996; the paper names
interior-point methods without fixing one).  Primal X with diag(X) = 1 and
dual y with Z = T - Diag(y) positive definite stay feasible throughout; each
iteration targets sigma mu (mu = <X, Z>/N) on the central path:
    (X o Z^-1) dy = 1 - sigma mu diag(Z^-1)          (o: elementwise product)
    dZ = -Diag(dy),   dX = sigma mu Z^-1 - X + X Diag(dy) Z^-1 (symmetrised)
with step lengths 0.95 of the largest keeping X and Z positive definite
(from the eigenvalues of L^-1 dX L^-T).  The iteration ends at a relative
gap of ``tol``, or earlier when X or Z no longer admits a Cholesky
factorisation in float64 (a degenerate problem whose gap has reached the
rounding floor; ``gap`` reports where it stopped).  Readings where the paper is
silent: T is scaled by 1 / max|T_ij| for the solve (the argmin does not
change); the eigenvector is oriented so that its last entry, the
coordinate of the fixed 1 in s~, is non-negative; sign(0) = +1.
"""
from __future__ import annotations

import numpy as np


def solve_sdr(T, tol=1e-10, sigma=0.2, max_iter=200):
    """Solve eq. (7) for one symmetric T [N, N].  Returns dict X, y, Z,
    objective = Tr(T X), dual = sum(y) (both in the units of T), gap =
    <X, Z> (scaled units), iterations."""
    T = np.asarray(T, dtype=np.float64)
    N = T.shape[0]
    scale = np.max(np.abs(T))
    if scale == 0.0:
        return {"X": np.eye(N), "y": np.zeros(N), "Z": np.zeros((N, N)), "objective": 0.0,
                "dual": 0.0, "gap": 0.0, "iterations": 0}
    C = T / scale
    X = np.eye(N)
    # a diagonally dominant, hence positive definite, starting Z
    y = np.diag(C) - np.sum(np.abs(C), axis=1) + np.abs(np.diag(C)) - 1.0
    Z = C - np.diag(y)
    it = 0
    for it in range(1, max_iter + 1):
        mu = np.sum(X * Z) / N
        if np.sum(X * Z) <= tol * max(1.0, abs(np.sum(C * X))):
            break
        Zi = np.linalg.inv(Z)
        Zi = 0.5 * (Zi + Zi.T)
        M = X * Zi
        dy = np.linalg.solve(M, 1.0 - sigma * mu * np.diag(Zi))
        dX = sigma * mu * Zi - X + X @ np.diag(dy) @ Zi
        dX = 0.5 * (dX + dX.T)
        dZ = -np.diag(dy)
        try:
            ap = _max_step(X, dX)
            ad = _max_step(Z, dZ)
        except np.linalg.LinAlgError:
            break                                     # X or Z no longer factors: rounding floor reached
        X = X + min(1.0, 0.95 * ap) * dX
        y = y + min(1.0, 0.95 * ad) * dy
        Z = C - np.diag(y)
    return {"X": X, "y": y * scale, "Z": Z * scale, "objective": float(np.sum(T * X)),
            "dual": float(np.sum(y) * scale), "gap": float(np.sum(X * Z)), "iterations": it}


def _max_step(P, dP):
    """Largest alpha with P + alpha dP positive semidefinite (P positive
    definite): 1 / max(0, -lambda_min(L^-1 dP L^-T)) with P = L L^T."""
    L = np.linalg.cholesky(P)
    W = np.linalg.solve(L, np.linalg.solve(L, dP).T)
    lam = np.linalg.eigvalsh(0.5 * (W + W.T)).min()
    return np.inf if lam >= 0 else -1.0 / lam


def round_leading_eigenvector(X):
    """Signs of the leading eigenvector of X (Section II-C), oriented so that
    the last entry (the fixed 1 of s~) is non-negative.  Returns (sbar for
    the first N-1 entries, the eigenvector u, its eigenvalues in
    decreasing order)."""
    w, V = np.linalg.eigh(np.asarray(X, dtype=np.float64))
    u = V[:, -1]
    if u[-1] < 0:
        u = -u
    sbar = np.where(u[:-1] >= 0, 1, -1).astype(np.int8)
    return sbar, u, w[::-1]


def sdr_detect(T):
    """The exact SDR detector for a batch T [V, N, N]: per vector the SDP
    solution and its rounding.  Returns dict sbar [V, N-1], objective [V],
    dual [V], u [V, N] (leading eigenvectors), eig [V, N] (eigenvalues of
    S^, decreasing), X [V, N, N]."""
    T = np.asarray(T, dtype=np.float64)
    V, N, _ = T.shape
    out = {"sbar": np.zeros((V, N - 1), dtype=np.int8), "objective": np.zeros(V), "dual": np.zeros(V),
           "u": np.zeros((V, N)), "eig": np.zeros((V, N)), "X": np.zeros((V, N, N))}
    for v in range(V):
        r = solve_sdr(T[v])
        sb, u, w = round_leading_eigenvector(r["X"])
        out["sbar"][v], out["u"][v], out["eig"][v], out["X"][v] = sb, u, w, r["X"]
        out["objective"][v], out["dual"][v] = r["objective"], r["dual"]
    return out
