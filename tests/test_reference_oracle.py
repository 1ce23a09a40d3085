"""Pins of the reference-detector oracle (oracle/reference.py): the paper's
comparison detectors (Section V-A) against closed forms, other library
routines, brute force and cases worked by hand."""
import numpy as np
import pytest

import oracle
import sim
from oracle import ml, reference


def _mimo(B, U, mod, V, snr, seed, noiseless=False):
    d = sim.gen_mimo(B, U, mod, V, 1, snr, seed, noiseless=noiseless)
    return d["H"], d["y"], d["s"], d["N0"]


def _sbar_of(s, mod):
    s = np.asarray(s)
    return np.concatenate([s.real, s.imag], axis=-1) if mod == oracle.QPSK else s.real


@pytest.mark.parametrize("mod", [oracle.QPSK, oracle.BPSK])
def test_matched_filter_is_one_taser_iteration_and_complex_form(mod):
    """The matched filter's signs are Algorithm 1's after one iteration
    (from L~(0) = D) and those of Re/Im of H^H y computed in complex."""
    H, y, _, _ = _mimo(24, 6, mod, 300, 2.0, 501)
    sb, x = reference.matched_filter(H, y, mod)
    t1 = oracle.detect_coherent(H, y, mod, alpha=0.5, t_max=1)
    np.testing.assert_array_equal(sb, t1["sbar"])
    mf = np.einsum("vbu,vb->vu", np.conj(H.astype(np.complex128)), y.astype(np.complex128))
    np.testing.assert_allclose(x, _sbar_of(mf, mod), rtol=1e-12, atol=1e-12)


def test_mmse_complex_form_and_limits():
    """QPSK: the real-valued MMSE equals the complex (H^H H + (N0/2) I)^-1
    H^H y split into real and imaginary parts; as N0 -> 0 it becomes least
    squares (LAPACK's lstsq, a different routine) on a tall channel; as
    N0 -> infinity its signs become the matched filter's."""
    mod = oracle.QPSK
    H, y, _, n0 = _mimo(20, 6, mod, 100, 3.0, 502)
    _, x = reference.mmse(H, y, mod, n0)
    Hc, yc = H.astype(np.complex128), y.astype(np.complex128)
    G = np.conj(np.swapaxes(Hc, 1, 2)) @ Hc + (n0 / 2) * np.eye(6)
    xc = np.linalg.solve(G, np.einsum("vbu,vb->vu", np.conj(Hc), yc)[..., None])[..., 0]
    np.testing.assert_allclose(x, _sbar_of(xc, mod), rtol=1e-10, atol=1e-12)
    _, x0 = reference.mmse(H, y, mod, 1e-12)
    Hbar, ybar = oracle.real_decomposition_coherent(H, y, mod)
    ls = np.stack([np.linalg.lstsq(Hbar[v], ybar[v], rcond=None)[0] for v in range(100)])
    np.testing.assert_allclose(x0, ls, rtol=1e-7, atol=1e-9)
    sb_inf, _ = reference.mmse(H, y, mod, 1e12)
    np.testing.assert_array_equal(sb_inf, reference.matched_filter(H, y, mod)[0])


def test_kbest_worked_by_hand():
    """A 2-level real problem worked by hand: R = [[1, 0.5], [0, 0.2]],
    z = (0.1, 0.01).  Level 2: s_2 = +1 gives (0.01 - 0.2)^2 = 0.0361,
    s_2 = -1 gives 0.21^2 = 0.0441.  K = 1 keeps s_2 = +1, then s_1 = -1:
    0.0361 + (0.1 + 1 - 0.5)^2 = 0.3961.  K = 2 also extends s_2 = -1 with
    s_1 = +1: 0.0441 + (0.1 - 1 + 0.5)^2 = 0.2041, the ML path."""
    H = np.array([[[1.0, 0.5], [0.0, 0.2]]], dtype=np.complex128)     # BPSK, B = U = 2, real
    y = np.array([[0.1, 0.01]], dtype=np.complex128)
    sb1, m1 = reference.kbest(H, y, oracle.BPSK, 1)
    sb2, m2 = reference.kbest(H, y, oracle.BPSK, 2)
    np.testing.assert_array_equal(sb1[0], [-1, 1])
    np.testing.assert_array_equal(sb2[0], [1, -1])
    assert abs(m1[0] - 0.3961) < 1e-12 and abs(m2[0] - 0.2041) < 1e-12
    s_ml, c_ml = ml.ml_coherent(H, y, oracle.BPSK)
    np.testing.assert_array_equal(sb2[0], s_ml[0].real.astype(np.int8))


@pytest.mark.parametrize("mod, U", [(oracle.BPSK, 4), (oracle.QPSK, 2)])
def test_kbest_keeping_every_path_is_ml(mod, U):
    """With K >= 2^(N-1) no path is ever dropped, so K-best is exhaustive:
    its decision is the ML decision of eq. (1) (complex brute force) and its
    metric plus the part of ybar outside the range of Hbar is the ML cost."""
    H, y, _, _ = _mimo(6, U, mod, 80, 0.0, 503)
    M = 2 * U if mod == oracle.QPSK else U
    sb, metric = reference.kbest(H, y, mod, 2 ** M)
    s_ml, cost = ml.ml_coherent(H, y, mod)
    np.testing.assert_array_equal(sb, _sbar_of(s_ml, mod).astype(np.int8))
    Hbar, ybar = oracle.real_decomposition_coherent(H, y, mod)
    Q = np.linalg.qr(Hbar)[0]
    outside = np.sum(ybar ** 2, axis=-1) - np.sum(np.einsum("vbm,vb->vm", Q, ybar) ** 2, axis=-1)
    np.testing.assert_allclose(metric + outside, cost, rtol=1e-10)
    np.testing.assert_allclose(reference.residual(H, y, mod, sb), cost, rtol=1e-10)


def test_kbest_bounds_and_noiseless_recovery():
    """K = 5 never beats ML (its residual >= the ML cost), and on a noiseless
    tall channel it recovers the transmitted symbols with a residual at the
    rounding level of the complex64 inputs."""
    H, y, _, _ = _mimo(8, 4, oracle.QPSK, 120, -2.0, 504)
    sb, _ = reference.kbest(H, y, oracle.QPSK, 5)
    _, cost = ml.ml_coherent(H, y, oracle.QPSK)
    assert np.all(reference.residual(H, y, oracle.QPSK, sb) >= cost * (1 - 1e-12))
    H, y, s, _ = _mimo(32, 8, oracle.QPSK, 50, 0.0, 505, noiseless=True)
    sb, metric = reference.kbest(H, y, oracle.QPSK, 5)
    np.testing.assert_array_equal(sb, _sbar_of(s, oracle.QPSK).astype(np.int8))
    # the inputs are stored as complex64: the residual is their rounding only
    assert metric.max() < 1e-8
