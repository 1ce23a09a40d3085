"""Scalar, multiplication-counting restatement of Algorithm 1 (test only).

The loop performs Algorithm 1 entry by entry, the way the systolic array of
Section IV-A schedules it: the product L~ T^ skips the terms that are zero
because L~ is lower triangular, each column's squared norm is a chain of
squares, one scale factor D_jj / ||v_j|| is formed per column, and every
entry of V is multiplied by its column's factor.  T^ = 2 tau T~ is formed in
preprocessing (Section IV-A) and is not counted, as Table I ignores
preprocessing.  The count must equal Table I's formula exactly.

It is an independent second implementation (pure Python floats, no numpy
linear algebra) used to pin the batched oracle on tiny inputs.
"""
from __future__ import annotations

import math


def taser_counted(Tt, D, tau, t_max, pin_last=False):
    """Returns (L as a list of lists, number of real multiplications).

    pin_last=False is the literal Algorithm 1 (every column normalised),
    which is what Table I counts."""
    N = len(D)
    That = [[2.0 * tau * Tt[k][j] for j in range(N)] for k in range(N)]  # preprocessing
    L = [[(D[i] if i == j else 0.0) for j in range(N)] for i in range(N)]
    mults = 0
    for _ in range(t_max):
        V = [[0.0] * N for _ in range(N)]
        for i in range(N):
            for j in range(i + 1):
                acc = L[i][j]
                for k in range(i + 1):           # L~_{i,k} = 0 for k > i
                    acc -= L[i][k] * That[k][j]
                    mults += 1
                V[i][j] = acc
        scale = [0.0] * N
        for j in range(N):
            sq = 0.0
            for i in range(j, N):
                sq += V[i][j] * V[i][j]
                mults += 1
            scale[j] = D[j] * (1.0 / math.sqrt(sq))
            mults += 1
        for i in range(N):
            for j in range(i + 1):
                L[i][j] = V[i][j] * scale[j]
                mults += 1
        if pin_last:
            L[N - 1][N - 1] = D[N - 1]
    return L, mults
