"""Pins of the exact-SDR oracle (oracle/sdr.py, eq. (7)): a closed form at
N = 2, the optimality conditions of the SDP, an independent solver
(Burer-Monteiro low-rank factorisation), the relaxation bound against
exhaustive ML, and rank-one tightness on noiseless systems."""
import numpy as np
import pytest

import oracle
import sim
from oracle import ml, sdr


def test_two_by_two_closed_form():
    """N = 2: S = [[1, x], [x, 1]] with |x| <= 1, Tr(T S) = T11 + T22 + 2 T12 x,
    minimised at x = -sign(T12): T11 + T22 - 2 |T12| (by hand: 3 + 2 - 2.4)."""
    r = sdr.solve_sdr(np.array([[3.0, -1.2], [-1.2, 2.0]]))
    assert abs(r["objective"] - 2.6) < 1e-8
    np.testing.assert_allclose(r["X"], [[1.0, 1.0], [1.0, 1.0]], atol=1e-5)


def _mimo_T(B, U, mod, V, snr, seed, noiseless=False):
    d = sim.gen_mimo(B, U, mod, V, 1, snr, seed, noiseless=noiseless)
    return oracle.build_T_coherent(d["H"], d["y"], mod), d


@pytest.mark.parametrize("B, U, mod, snr", [(8, 3, oracle.QPSK, 0.0), (6, 5, oracle.BPSK, -3.0),
                                            (4, 4, oracle.QPSK, 5.0)])
def test_optimality_conditions_and_relaxation_bound(B, U, mod, snr):
    """Primal feasibility diag(S) = 1, S PSD; dual feasibility
    Z = T - Diag(y) PSD; weak duality sum(y) <= Tr(T S) with a vanishing
    gap; and the relaxation bound Tr(T S^) <= min over s~ of s~^T T s~
    (exhaustive ML over eq. (2))."""
    T, _ = _mimo_T(B, U, mod, 12, snr, 700 + B + U)
    _, ml_val = ml.ml_over_T(T)
    for v in range(T.shape[0]):
        r = sdr.solve_sdr(T[v])
        X, Z, scale = r["X"], r["Z"], np.abs(T[v]).max()
        np.testing.assert_allclose(np.diag(X), 1.0, atol=1e-10)
        assert np.linalg.eigvalsh(X).min() > -1e-10
        np.testing.assert_allclose(Z, T[v] - np.diag(r["y"]), atol=1e-9 * scale)
        assert np.linalg.eigvalsh(Z).min() > -1e-8 * scale
        assert r["dual"] <= r["objective"] + 1e-9 * scale
        assert r["objective"] - r["dual"] < 1e-7 * scale * T.shape[-1]
        assert r["objective"] <= ml_val[v] * (1 + 1e-8) + 1e-9 * scale


def _burer_monteiro(T, p, iters=20000, seed=0):
    """min Tr(T V V^T) over V [N, p] with unit rows, by projected gradient on
    the product of spheres; for p(p+1)/2 > N its second-order critical points
    are global minima of the SDP (an independent route to the optimum)."""
    N = T.shape[0]
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((N, p))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    C = T / np.abs(T).max()
    lr = 0.5 / np.linalg.norm(C, 2)
    for _ in range(iters):
        G = 2.0 * C @ V
        G -= np.sum(G * V, axis=1, keepdims=True) * V
        V -= lr * G
        V /= np.linalg.norm(V, axis=1, keepdims=True)
    return float(np.sum(C * (V @ V.T)) * np.abs(T).max())


def test_agrees_with_burer_monteiro():
    T, _ = _mimo_T(10, 4, oracle.QPSK, 4, 2.0, 711)
    for v in range(T.shape[0]):
        r = sdr.solve_sdr(T[v])
        bm = _burer_monteiro(T[v], p=5)
        assert abs(bm - r["objective"]) <= 1e-7 * abs(r["objective"])


def test_rank_one_on_noiseless_tall_systems():
    """Without noise on a tall channel s~ s~^T is optimal (Tr(T S) = 0 there
    and T is PSD): the relaxation is tight, S^ has rank one and the rounding
    returns the transmitted symbols, with the last eigenvector entry
    oriented non-negative."""
    T, d = _mimo_T(16, 4, oracle.QPSK, 8, 0.0, 712, noiseless=True)
    out = sdr.sdr_detect(T)
    truth = np.concatenate([d["s"].real, d["s"].imag], axis=1).astype(np.int8)
    np.testing.assert_array_equal(out["sbar"], truth)
    assert np.all(out["eig"][:, 1] < 1e-6 * out["eig"][:, 0])
    assert np.all(out["u"][:, -1] >= 0)
    assert np.all(np.abs(out["objective"]) < 1e-6 * np.abs(T).max(axis=(1, 2)))


def test_joint_detection_matrix():
    """eq. (5)'s T is negative semidefinite; the SDP is the same program: the
    relaxation bound against exhaustive ML over that T holds."""
    d = sim.gen_jed(8, 4, oracle.QPSK, 6, 2.0, 713)
    T = oracle.build_T_jed(d["Y"], d["s0"], oracle.QPSK)
    _, ml_val = ml.ml_over_T(T)
    out = sdr.sdr_detect(T)
    assert np.all(out["objective"] <= ml_val + 1e-8 * np.abs(ml_val))
