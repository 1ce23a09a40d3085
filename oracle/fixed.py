"""Fixed-point TASER in plain integer numpy (test infrastructure only).

Algorithm 1 in the 14-bit fixed-point arithmetic of the paper's hardware
(Section IV-C, "Fixed-point design parameters" and "Inverse square-root
computation"), given the preprocessed inputs T^ = 2 tau T~ and D of
Section IV-A.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use this module; it shares no code with
the HIP path.

What the paper fixes:
  * every word is a 14-bit number;
  * L~ and V use 8 fraction bits, except the bottom row of the triangular
    array (row N), which uses 7;
  * L~_NN is not a processing element: it is held constant in a register
    with 5 fraction bits;
  * the inverse square root of the squared column norm comes from a table of
    2^11 words of 14 bits with 13 fraction bits, and the scale unit
    multiplies it by D_jj.

Readings where the paper is silent (Q1..Q8, also listed in the design
notes):
  Q1 words are two's complement and saturate at [-2^13, 2^13 - 1];
  Q2 T^ = 2 tau T~ has 12 fraction bits (|T~_ij| <= 1 and tau <= 1/||T~||_2
     <= 1, so |T^_ij| < 2 fits); D_kk (k < N) has the 8 fraction bits of the
     diagonal element it initialises, D_NN the 5 of L~_NN;
  Q3 a processing element accumulates its products exactly (a wide
     accumulator) and rounds once, when V_ij is stored;
  Q4 rounding is to nearest with ties upwards: floor(x / 2^s + 1/2);
  Q5 squared column norms are exact sums, with 16 fraction bits (the bottom
     row's 7-bit values are aligned by 2^2 before squaring);
  Q6 the table is indexed by the top 11 bits of the squared norm after a
     shift by an even number of bits that puts its leading one in bit 10 or
     9 (so indices 512..2047 occur), and entry i holds the integer nearest
     to 2^13 / sqrt((i + 1/2) / 2^10);
  Q7 the scale factor D_jj / ||v_j|| has 11 fraction bits;
  Q8 a column whose squared norm is 0 is reset to D_jj e_j (reading R8 of
     the floating-point oracle), and vectors flagged degenerate or
     non-finite by the preprocessing run no iterations.
"""
from __future__ import annotations

import math

import numpy as np

WORD_BITS = 14
WMIN, WMAX = -(1 << (WORD_BITS - 1)), (1 << (WORD_BITS - 1)) - 1
F_L = 8        # L~ and V, rows 1..N-1 (and D_kk, k < N)
F_B = 7        # bottom row of L~ and V
F_NN = 5       # L~_NN = D_NN
F_T = 12       # T^ = 2 tau T~ (reading Q2)
F_Q = 16       # squared column norms (reading Q5)
F_C = 11       # scale factor D_jj / ||v_j|| (reading Q7)
LUT_BITS = 11
LUT_FRAC = 13

VEC_ZERO_NORM = 4


def quantize(x, frac_bits):
    """Real value -> 14-bit word with ``frac_bits`` fraction bits (Q1, Q4)."""
    q = np.floor(np.asarray(x, dtype=np.float64) * float(1 << frac_bits) + 0.5)
    return np.clip(q, WMIN, WMAX).astype(np.int64)


def round_shift(x, s):
    """floor(x / 2^s + 1/2) for int64 x and s >= 1 (Q4)."""
    return (np.asarray(x, dtype=np.int64) + (1 << (s - 1))) >> s


def saturate(x):
    return np.clip(x, WMIN, WMAX)


def rsqrt_table():
    """The 2^11-word inverse-square-root table (Q6): entry i (i >= 512) is the
    integer nearest to 2^13 / sqrt((i + 1/2) / 2^10) = 2^18 / sqrt(i + 1/2),
    found exactly with integer arithmetic: r is nearest to sqrt(X) with
    X = 2^37 / (2i + 1) iff (2r - 1)^2 (2i + 1) <= 2^39 < (2r + 1)^2 (2i + 1)
    (equality cannot occur: the left side is odd).  Entries below 512 are
    never indexed and hold 0."""
    lut = np.zeros(1 << LUT_BITS, dtype=np.int64)
    for i in range(1 << (LUT_BITS - 2), 1 << LUT_BITS):
        m = 2 * i + 1
        r = math.isqrt((1 << 37) // m)          # within one of the answer
        while (2 * r + 1) ** 2 * m <= (1 << 39):
            r += 1
        while (2 * r - 1) ** 2 * m > (1 << 39):
            r -= 1
        lut[i] = r
    return lut


_LUT = None


def _lut():
    global _LUT
    if _LUT is None:
        _LUT = rsqrt_table()
    return _LUT


def scale_factor(q, d):
    """The scale unit (Section IV-A): D_jj / ||v_j|| with 11 fraction bits,
    from the squared norm q (> 0, 16 fraction bits) and D_jj (8 fraction
    bits), via the table (Q6, Q7).  With q = idx 2^s (s even),
    1/sqrt(q 2^-16) = LUT[idx] 2^(-10 - s/2), so the factor in units of
    2^-11 is d LUT[idx] 2^(-7 - s/2)."""
    q = np.asarray(q, dtype=np.int64)
    d = np.asarray(d, dtype=np.int64)
    lut = _lut()
    out = np.zeros(np.broadcast(q, d).shape, dtype=np.int64)
    qf = np.broadcast_to(q, out.shape).ravel()
    df = np.broadcast_to(d, out.shape).ravel()
    of = out.ravel()
    for n in range(qf.size):
        qq = int(qf[n])
        p = qq.bit_length()
        s = p - LUT_BITS
        if s % 2:
            s += 1
        idx = qq >> s if s >= 0 else qq << (-s)
        shift = 7 + s // 2
        v = (int(df[n]) * int(lut[idx]) + (1 << (shift - 1))) >> shift
        of[n] = min(max(v, 0), WMAX)
    return out


def fixed_inputs(Tt, D, tau, product_dtype=np.float64):
    """Quantise the preprocessing outputs (Q2): T^ = 2 tau T~ with 12
    fraction bits; D_kk with 8 (k < N) and D_NN with 5 fraction bits.
    ``product_dtype`` is the precision in which 2 tau T~ is formed before
    rounding to a word: float64 here, float32 to take the same decision as a
    float32 preprocessing does (2 tau is exact in either; the product is
    rounded once)."""
    Tt = np.asarray(Tt, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    two_tau = (2.0 * tau).astype(product_dtype)[..., None, None]
    prod = (two_tau * Tt.astype(product_dtype)).astype(np.float64)
    That = quantize(prod, F_T)
    d = quantize(D, F_L)
    d[..., -1] = quantize(D[..., -1], F_NN)
    return That, d


def fixed_iterate(That, d, t_max, skip=None):
    """Algorithm 1 in fixed point.  That [V, N, N] (12 fraction bits), d [V, N]
    (D_kk, 8 fraction bits; D_NN, 5).  Returns (L, status): L [V, N, N] int64
    words, rows 1..N-1 with 8 fraction bits, row N with 7 (L~_NN as its
    5-bit register value), and status bits (VEC_ZERO_NORM).

    Each iteration, for every element j <= i of row i (row format F):
        acc   = L_ij 2^12 - sum_{k <= i} L_ik T^_kj      (exact, Q3)
        V_ij  = sat(round(acc / 2^12))                  (F fraction bits)
    then for every column j < N the squared norm
        q_j = sum_{i < N} V_ij^2 + 4 V_Nj^2             (16 fraction bits, Q5)
    and, with the scale unit's c_j (Q6, Q7),
        L_ij = sat(round(V_ij c_j / 2^11))              (same row format)
    while L~_NN keeps its 5-bit value (Section IV-C)."""
    That = np.asarray(That, dtype=np.int64)
    d = np.asarray(d, dtype=np.int64)
    V_, N, _ = That.shape
    status = np.zeros(V_, dtype=np.int32)
    L = np.zeros((V_, N, N), dtype=np.int64)
    idx = np.arange(N - 1)
    L[:, idx, idx] = d[:, :N - 1]
    lnn = d[:, N - 1]
    L[:, N - 1, N - 1] = lnn
    skip = np.zeros(V_, dtype=bool) if skip is None else np.asarray(skip, dtype=bool)
    run = ~skip
    tril = np.tril(np.ones((N, N), dtype=bool))
    for _ in range(t_max):
        # the bottom row's arithmetic uses L~_NN aligned to its 7 fraction bits
        Lw = L.copy()
        Lw[:, N - 1, N - 1] = lnn << (F_B - F_NN)
        P = np.matmul(Lw, That)                       # exact int64 sums over k <= i
        acc = (Lw << F_T) - P
        V = saturate(round_shift(acc, F_T))
        V = np.where(tril, V, 0)
        sq = V[:, :N - 1, :N - 1] ** 2
        q = sq.sum(axis=1) + (V[:, N - 1, :N - 1] ** 2) * (1 << (2 * (F_L - F_B)))
        zero = q == 0
        c = np.zeros_like(q)
        nz = ~zero & run[:, None]
        if np.any(nz):
            c[nz] = scale_factor(q[nz], d[:, :N - 1][nz])
        Lnew = saturate(round_shift(V[:, :, :N - 1] * c[:, None, :], F_C))
        if np.any(zero):
            reset = np.zeros((V_, N, N - 1), dtype=np.int64)
            reset[:, idx, idx] = d[:, :N - 1]
            Lnew = np.where(zero[:, None, :], reset, Lnew)
            status |= np.where(np.any(zero, axis=1) & run, VEC_ZERO_NORM, 0).astype(np.int32)
        Lnext = np.zeros_like(L)
        Lnext[:, :, :N - 1] = Lnew
        Lnext[:, N - 1, N - 1] = lnn
        L = np.where(run[:, None, None], Lnext, L)
    return L, status


def fixed_decisions(L):
    """Algorithm 1 output on the bottom row: sbar_k = sign(L~_Nk), sign(0) = +1."""
    last = np.asarray(L)[..., -1, :-1]
    return np.where(last >= 0, 1, -1).astype(np.int8)


def to_real(L):
    """Words -> real values (rows 1..N-1: 8 fraction bits, row N: 7, L~_NN: 5)."""
    L = np.asarray(L, dtype=np.float64)
    N = L.shape[-1]
    out = L / float(1 << F_L)
    out[..., N - 1, :] = L[..., N - 1, :] / float(1 << F_B)
    out[..., N - 1, N - 1] = L[..., N - 1, N - 1] / float(1 << F_NN)
    return out
