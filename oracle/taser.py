"""Plain FP64 CPU TASER, written from the paper (test infrastructure only).

Castaneda, Goldstein and Studer, "Data Detection in Large Multi-Antenna
Wireless Systems via Approximate Semidefinite Relaxation", arXiv:1609.01797.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It shares no code with the HIP path and
imports nothing from it.  Inputs are the complex64 arrays the GPU reads,
upcast to complex128; all arithmetic is float64.

Every function is batched over leading axes with plain numpy (stacked
matmul, tril, sums); there is no blocking, fusion or reordering beyond the
paper's own steps.  Where the paper is silent or ambiguous the reading used
is stated at the function (readings R1..R11, listed in the design notes).
"""
from __future__ import annotations

import numpy as np

BPSK = 1
QPSK = 2
COHERENT = 0
JED = 1

# per-vector status bits (same meaning as the library's)
VEC_DEGENERATE = 1   # some T_kk == 0: no iterations are run
VEC_NONFINITE = 2    # NaN / Inf in the inputs: no iterations are run
VEC_ZERO_NORM = 4    # a prox column had zero (or non-finite) norm; reset applied
VEC_VNN_NONPOS = 8   # V_NN <= 0 occurred (diagnostic for the pinned corner)


def problem_size(U: int, mod: int) -> int:
    """N = 2U+1 for QPSK, U+1 for BPSK (Section II-A, below eq. (2))."""
    return 2 * U + 1 if mod == QPSK else U + 1


# ----------------------------------------------------------------------------
# Section II: real-valued reformulation
# ----------------------------------------------------------------------------

def real_decomposition_coherent(H, y, mod):
    """Section II-A.  ybar = [Re y; Im y].
    QPSK: Hbar = [[Re H, -Im H], [Im H, Re H]]  (2B x 2U).
    BPSK: underline H = [Re H; Im H]            (2B x U).
    H: [..., B, U], y: [..., B]."""
    H = np.asarray(H).astype(np.complex128)
    y = np.asarray(y).astype(np.complex128)
    ybar = np.concatenate([y.real, y.imag], axis=-1)
    if mod == QPSK:
        top = np.concatenate([H.real, -H.imag], axis=-1)
        bot = np.concatenate([H.imag, H.real], axis=-1)
        Hbar = np.concatenate([top, bot], axis=-2)
    elif mod == BPSK:
        Hbar = np.concatenate([H.real, H.imag], axis=-2)
    else:
        raise ValueError(mod)
    return Hbar, ybar


def build_T_coherent(H, y, mod):
    """eq. (2): T = [Hbar^T Hbar, -Hbar^T ybar; -ybar^T Hbar, ybar^T ybar].

    Formed literally as A^T A with A = [Hbar, -ybar] from the 2B-row real
    matrices (the same matrix, since (A s~) = Hbar sbar - ybar)."""
    Hbar, ybar = real_decomposition_coherent(H, y, mod)
    A = np.concatenate([Hbar, -ybar[..., :, None]], axis=-1)
    return np.swapaxes(A, -1, -2) @ A


def real_decomposition_jed(Y, s0, mod):
    """Section II-B.  Y: [..., K+1, B] slot-major (Y[..., k, :] is y_k),
    s0: [...] known first entry of the paper's s.
    ybar = [Re(y0 s0); Im(y0 s0)]; Hbar (QPSK) or underline H (BPSK) is built
    from Y_r = [y_1, ..., y_K] exactly as H is in the coherent case."""
    Y = np.asarray(Y).astype(np.complex128)
    s0 = np.asarray(s0).astype(np.complex128)
    y0s0 = Y[..., 0, :] * s0[..., None]
    Yr = np.swapaxes(Y[..., 1:, :], -1, -2)          # [..., B, K]
    Hbar, ybar = real_decomposition_coherent(Yr, y0s0, mod)
    return Hbar, ybar


def build_T_jed(Y, s0, mod):
    """eq. (5): T = -[Hbar^T Hbar, Hbar^T ybar; ybar^T Hbar, ybar^T ybar],
    i.e. T = -A^T A with A = [Hbar, ybar]."""
    Hbar, ybar = real_decomposition_jed(Y, s0, mod)
    A = np.concatenate([Hbar, ybar[..., :, None]], axis=-1)
    return -(np.swapaxes(A, -1, -2) @ A)


# ----------------------------------------------------------------------------
# Section III-B / III-C: step size and Jacobi preconditioning
# ----------------------------------------------------------------------------

def precondition(T):
    """Section III-C: D = diag(sqrt(T_kk)), T~ = D^-1 T D^-1.

    Reading R3: the joint-detection T of eq. (5) is negative semidefinite, so
    sqrt(T_kk) is taken of |T_kk|; T~ then has diagonal -1 instead of +1.
    Returns (D [..., N], Tt [..., N, N], degenerate [...] bool).  Degenerate
    vectors (some T_kk == 0) get D = 1 and T~ = 0 rows so the arithmetic
    stays finite; their results are overridden by ``run_taser``."""
    T = np.asarray(T, dtype=np.float64)
    d = np.abs(np.diagonal(T, axis1=-2, axis2=-1))
    degenerate = np.any(d == 0.0, axis=-1)
    D = np.sqrt(np.where(d == 0.0, 1.0, d))
    Tt = T / (D[..., :, None] * D[..., None, :])
    return D, Tt, degenerate


def spectral_norm(Tt):
    """||T~||_2 of the symmetric T~ (Section III-B): the largest |eigenvalue|,
    from LAPACK's symmetric eigensolver."""
    ev = np.linalg.eigvalsh(np.asarray(Tt, dtype=np.float64))
    return np.max(np.abs(ev), axis=-1)


def step_size(Tt, alpha):
    """tau = alpha / ||T~||_2 (Algorithm 1 inputs; Section III-B).
    Reading R5: the norm is taken of the preconditioned T~, as Algorithm 1 and
    the remark after Proposition 1 state."""
    return np.asarray(alpha, dtype=np.float64) / spectral_norm(Tt)


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------

def objective(L, Tt):
    """f(L~) = Tr(L~ T~ L~^T) (eq. (8), preconditioned)."""
    return np.trace(L @ Tt @ np.swapaxes(L, -1, -2), axis1=-2, axis2=-1)


def taser_iterate(Tt, D, tau, t_max, pin_last=True, record=False, L0=None,
                  per_iteration=False):
    """Algorithm 1, initialisation and main loop.

    Tt: [..., N, N], D: [..., N], tau: scalar or [...]; with
    per_iteration=True, tau is [t_max, ...] (one step size per iteration, the
    unfolded variant; a constant step size is the paper's algorithm).

      L~(0) = D
      for t = 1..t_max:
        V(t)  = L~(t-1) - tril(2 tau L~(t-1) T~)
        L~(t) = prox(V(t)):  column k <- D_kk V_:,k / ||V_:,k||_2

    Reading R1: the prox rescales the COLUMNS of L~ (Section III-A constrains
    the k-th column; Section III-C rescales the k-th column by D_kk).
    Reading R6 (pin_last=True, default): L~_NN is held at D_NN, the
    projection onto the constraint set with a non-negative Cholesky diagonal
    (Section III-A), as the hardware does (Section IV-C stores L~_NN in a
    constant register).  pin_last=False is the literal normalisation, which
    gives D_NN * sign(V_NN).
    Reading R8: a column whose norm is zero or non-finite is reset to
    D_kk e_k (status VEC_ZERO_NORM).

    Returns (L, status) or (L, status, trace) with trace = dict of per-
    iteration objectives when record=True.
    """
    Tt = np.asarray(Tt, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    N = Tt.shape[-1]
    batch = Tt.shape[:-2]
    tau = np.asarray(tau, dtype=np.float64)
    status = np.zeros(batch, dtype=np.int32)
    eye = np.eye(N)
    L = (D[..., :, None] * eye) if L0 is None else np.array(L0, dtype=np.float64)
    objs = [objective(L, Tt)] if record else None
    for t in range(t_max):
        tau_t = tau[t] if per_iteration else tau
        tau_t = np.asarray(tau_t, dtype=np.float64)[..., None, None]
        V = L - np.tril(2.0 * tau_t * (L @ Tt))
        norms = np.sqrt(np.sum(V * V, axis=-2))                 # column norms
        bad = ~(np.isfinite(norms) & (norms > 0.0))
        safe = np.where(bad, 1.0, norms)
        if pin_last:
            bad[..., N - 1] = False
        status |= np.where(np.any(bad, axis=-1), VEC_ZERO_NORM, 0).astype(np.int32)
        status |= np.where(V[..., N - 1, N - 1] <= 0.0, VEC_VNN_NONPOS, 0).astype(np.int32)
        L = V * (D / safe)[..., None, :]
        if np.any(bad):
            reset = D[..., :, None] * eye
            L = np.where(bad[..., None, :], reset, L)
        if pin_last:
            L[..., N - 1, N - 1] = D[..., N - 1]
        if record:
            objs.append(objective(L, Tt))
    if record:
        return L, status, {"objective": np.stack(objs, axis=0)}
    return L, status


def slice_decisions(L, D):
    """Algorithm 1 output: sbar_k = sign(L~_{N,k}), k = 1..N-1.
    Reading R7: sign(0) = +1.  The margin L~_{N,k} / D_kk (the last row of the
    unpreconditioned L = L~ D^-1, a value in [-1, 1]) is returned with it."""
    L = np.asarray(L, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    last = L[..., -1, :-1]
    sbar = np.where(last >= 0.0, 1, -1).astype(np.int8)
    margin = last / D[..., :-1]
    return sbar, margin


def backmap(sbar, mod, U):
    """Section II-A: QPSK  s_i = sbar_i + j sbar_{i+U};  BPSK  s_i = sbar_i."""
    sbar = np.asarray(sbar).astype(np.float64)
    if mod == QPSK:
        return sbar[..., :U] + 1j * sbar[..., U:2 * U]
    return sbar[..., :U] + 0j


# ----------------------------------------------------------------------------
# Whole detectors
# ----------------------------------------------------------------------------

def _finite_complex(a, axes):
    a = np.asarray(a)
    return np.all(np.isfinite(a.real) & np.isfinite(a.imag), axis=axes)


def run_taser(T, alpha=None, t_max=10, tau=None, pin_last=True, record=False):
    """Preprocessing (Section III-C) + Algorithm 1 from a built T.

    Exactly one of ``alpha`` (tau = alpha/||T~||_2) and ``tau`` is given.
    Returns a dict: D, Tt, lam, tau, L, sbar, margin, status (+ trace).
    Degenerate or non-finite vectors (reading R8) run no iterations: L = D,
    decisions +1, margins 0."""
    T = np.asarray(T, dtype=np.float64)
    batch = T.shape[:-2]
    N = T.shape[-1]
    nonfinite = ~np.all(np.isfinite(T), axis=(-2, -1))
    Tc = np.where(nonfinite[..., None, None], 0.0, T)
    D, Tt, degenerate = precondition(Tc)
    lam = spectral_norm(Tt)
    if tau is None:
        lam_safe = np.where(lam > 0, lam, 1.0)
        tau_v = np.asarray(alpha, dtype=np.float64) / lam_safe
    else:
        tau_v = np.broadcast_to(np.asarray(tau, dtype=np.float64), batch) \
            if np.ndim(tau) <= len(batch) else np.asarray(tau, dtype=np.float64)
    skip = degenerate | nonfinite
    out = taser_iterate(Tt, D, tau_v, t_max, pin_last=pin_last, record=record)
    L, status = out[0], out[1]
    sbar, margin = slice_decisions(L, D)
    if np.any(skip):
        eye = np.eye(N)
        L = np.where(skip[..., None, None], D[..., :, None] * eye, L)
        sbar = np.where(skip[..., None], np.int8(1), sbar)
        margin = np.where(skip[..., None], 0.0, margin)
        status = np.where(skip, 0, status)
    status = status | np.where(degenerate & ~nonfinite, VEC_DEGENERATE, 0) \
        | np.where(nonfinite, VEC_NONFINITE, 0)
    res = {"D": D, "Tt": Tt, "lam": lam, "tau": tau_v, "L": L, "sbar": sbar,
           "margin": margin, "status": status.astype(np.int32)}
    if record:
        res["trace"] = out[2]
    return res


def detect_coherent(H, y, mod, alpha=None, t_max=10, tau=None, pin_last=True, record=False):
    """Coherent MU-MIMO detection (Section II-A + Algorithm 1).
    H: [..., B, U], y: [..., B] (broadcast H yourself for shared channels)."""
    T = build_T_coherent(H, y, mod)
    res = run_taser(T, alpha=alpha, t_max=t_max, tau=tau, pin_last=pin_last, record=record)
    U = np.asarray(H).shape[-1]
    res["T"] = T
    res["s_hat"] = backmap(res["sbar"], mod, U)
    return res


def detect_jed(Y, s0, mod, alpha=None, t_max=20, tau=None, pin_last=True, record=False):
    """SIMO joint channel estimation and detection (Section II-B + Algorithm 1).
    Y: [..., K+1, B] slot-major, s0: [...] pilot.  Returns the data symbols
    s_r (the paper's notation) and the channel estimate h = Y [s0; s_r]
    (eq. (4))."""
    T = build_T_jed(Y, s0, mod)
    res = run_taser(T, alpha=alpha, t_max=t_max, tau=tau, pin_last=pin_last, record=record)
    K = np.asarray(Y).shape[-2] - 1
    s_r = backmap(res["sbar"], mod, K)
    s_full = np.concatenate([np.asarray(s0).astype(np.complex128)[..., None], s_r], axis=-1)
    Yc = np.asarray(Y).astype(np.complex128)
    res["T"] = T
    res["s_hat"] = s_r
    res["h_hat"] = np.einsum("...kb,...k->...b", Yc, s_full)
    return res
