"""The Lanczos step count the kernels use for ||T~||_2 (Section III-C's step
size tau = alpha / ||T~||_2), checked on the CPU against the oracle's T~ and
LAPACK: min(N, 12 + N/8) steps for QPSK and min(N, 16 + N/4) for BPSK, from
the start T~ e_N and never past the dimension of its Krylov space (B complex
or 2B real dimensions), reach 1e-6 relative error on the spectra that need
the most steps.  The Lanczos here runs in float64 with full
reorthogonalisation, so it measures the Krylov space itself, not the
kernels' rounding (the GPU tests cover that)."""
import numpy as np
import pytest

import oracle
import sim


def steps_rule(N, B, qpsk):
    """Mirror of the kernels' step count (spectral::lanczos_steps, capped at
    the Krylov dimension of T~ e_N as the per-vector kernel does)."""
    m = 12 + N // 8 if qpsk else 16 + N // 4
    kdim = min(B, (N + 1) // 2) if qpsk else min(2 * B, N)
    return min(m, N, kdim)


def top_ritz(A, m):
    q = A[:, -1] / np.linalg.norm(A[:, -1])
    Q, al, be = [q], [], []
    for j in range(m):
        w = A @ Q[-1]
        al.append(Q[-1] @ w)
        for _ in range(2):
            M = np.array(Q)
            w = w - M.T @ (M @ w)
        b = np.linalg.norm(w)
        if j == m - 1 or b <= 1e-12 * max(abs(x) for x in al):
            break
        be.append(b)
        Q.append(w / b)
    T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    return np.linalg.eigvalsh(T)[-1]


CASES = [
    # (kind, B, U or K, mod, snr)
    ("coh", 64, 32, oracle.BPSK, 4.0),      # N = 33, U near B: N distinct eigenvalues
    ("coh", 32, 32, oracle.BPSK, -4.0),
    ("coh", 128, 64, oracle.BPSK, -4.0),    # N = 65 (staged path)
    ("coh", 128, 32, oracle.QPSK, -4.0),    # N = 65
    ("coh", 96, 64, oracle.QPSK, 0.0),      # N = 129
    ("jed", 16, 16, oracle.QPSK, -14.0),    # noise-dominated joint detection
    ("jed", 16, 16, oracle.BPSK, -14.0),
    ("jed", 4, 16, oracle.BPSK, 0.0),       # rank-deficient T~
]


@pytest.mark.parametrize("kind, B, U, mod, snr", CASES, ids=lambda x: str(x))
def test_lanczos_steps_reach_float32_resolution(kind, B, U, mod, snr):
    if kind == "coh":
        d = sim.gen_mimo(B, U, mod, 48, 1, snr, sim.seed_for(9, snr_index=int(snr) + 20, shard=U))
        T = oracle.build_T_coherent(d["H"], d["y"], mod)
        sg = 1.0
    else:
        d = sim.gen_jed(B, U, mod, 48, snr, sim.seed_for(9, snr_index=int(snr) + 40, shard=U))
        T = oracle.build_T_jed(d["Y"], d["s0"], mod)
        sg = -1.0
    _, Tt, _ = oracle.precondition(T)
    lam = oracle.spectral_norm(Tt)
    N = Tt.shape[1]
    m = steps_rule(N, B, mod == oracle.QPSK)
    rel = np.array([abs(top_ritz(sg * Tt[v], m) - lam[v]) / lam[v] for v in range(len(lam))])
    assert rel.max() <= 1e-6, (m, rel.max())


def test_fewer_steps_fall_short():
    """The same check fails with fewer steps: for BPSK with B = U = 32 at
    -4 dB, 12 steps (the earlier per-vector count) and 16 (what the QPSK rule
    would give at N = 33) both leave the top Ritz value more than 1e-5 short,
    so the test measures something and BPSK needs its longer rule."""
    d = sim.gen_mimo(32, 32, oracle.BPSK, 48, 1, -4.0, sim.seed_for(9, snr_index=16, shard=32))
    _, Tt, _ = oracle.precondition(oracle.build_T_coherent(d["H"], d["y"], oracle.BPSK))
    lam = oracle.spectral_norm(Tt)
    for m in (12, 16):
        rel = np.array([abs(top_ritz(Tt[v], m) - lam[v]) / lam[v] for v in range(len(lam))])
        assert rel.max() > 1e-5, (m, rel.max())
