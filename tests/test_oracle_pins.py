"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the
oracle's own formula: they use complex-valued objectives, brute force,
closed forms derived by hand, exact symmetries and Table I.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import sim
from oracle import ml
from oracle.counted import taser_counted

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mimo(B, U, mod, V, snr, seed, noiseless=False):
    d = sim.gen_mimo(B, U, mod, V, 1, snr, seed, noiseless=noiseless)
    return d["H"], d["y"], d["s"]


def _sbar_of(s, mod):
    s = np.asarray(s)
    if mod == oracle.QPSK:
        return np.concatenate([s.real, s.imag], axis=-1)
    return s.real


# ---------------------------------------------------------------- P1: eq. (2), eq. (5)

@pytest.mark.parametrize("mod,U", [(oracle.QPSK, 3), (oracle.BPSK, 5), (oracle.QPSK, 8)])
def test_T_identity_coherent(mod, U):
    """eq. (2): s~^T T s~ = ||y - H s||^2 for every s in O^U (Section II-A)."""
    H, y, _ = _mimo(12, U, mod, 20, 5.0, 11)
    T = oracle.build_T_coherent(H, y, mod)
    rng = np.random.default_rng(3)
    for _ in range(10):
        s = ml.constellation(mod)[rng.integers(0, 4 if mod == oracle.QPSK else 2, size=(20, U))]
        st = np.concatenate([_sbar_of(s, mod), np.ones((20, 1))], axis=1)
        lhs = np.einsum("vn,vnm,vm->v", st, T, st)
        rhs = np.sum(np.abs(y.astype(np.complex128) - np.einsum("vbu,vu->vb", H.astype(np.complex128), s)) ** 2, axis=1)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


@pytest.mark.parametrize("mod,K", [(oracle.QPSK, 3), (oracle.BPSK, 6)])
def test_T_identity_jed(mod, K):
    """eq. (5): s~^T T s~ = -||y0 s0 + Y_r s_r||^2 = -||Y s||^2 (Section II-B)."""
    d = sim.gen_jed(8, K, mod, 15, 5.0, 12)
    T = oracle.build_T_jed(d["Y"], d["s0"], mod)
    rng = np.random.default_rng(4)
    Yc = d["Y"].astype(np.complex128)
    for _ in range(10):
        sr = ml.constellation(mod)[rng.integers(0, 4 if mod == oracle.QPSK else 2, size=(15, K))]
        st = np.concatenate([_sbar_of(sr, mod), np.ones((15, 1))], axis=1)
        lhs = np.einsum("vn,vnm,vm->v", st, T, st)
        s_full = np.concatenate([d["s0"].astype(np.complex128)[:, None], sr], axis=1)
        rhs = -np.sum(np.abs(np.einsum("vkb,vk->vb", Yc, s_full)) ** 2, axis=1)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_T_is_symmetric_and_semidefinite():
    H, y, _ = _mimo(16, 4, oracle.QPSK, 10, 3.0, 13)
    T = oracle.build_T_coherent(H, y, oracle.QPSK)
    assert np.array_equal(T, np.swapaxes(T, 1, 2))
    assert np.all(np.linalg.eigvalsh(T) > -1e-9 * np.abs(T).max())
    d = sim.gen_jed(8, 4, oracle.QPSK, 10, 3.0, 13)
    Tj = oracle.build_T_jed(d["Y"], d["s0"], oracle.QPSK)
    assert np.all(np.linalg.eigvalsh(Tj) < 1e-9 * np.abs(Tj).max())


# ---------------------------------------------------------------- P2: brute-force ML

@pytest.mark.parametrize("mod,U", [(oracle.BPSK, 6), (oracle.QPSK, 3), (oracle.BPSK, 1)])
def test_ml_via_T_equals_complex_ml(mod, U):
    """eq. (1) and eq. (2) have the same minimiser (Section II-A)."""
    H, y, _ = _mimo(8, U, mod, 40, 0.0, 21)
    s_ml, _ = ml.ml_coherent(H, y, mod)
    T = oracle.build_T_coherent(H, y, mod)
    sbar, _ = ml.ml_over_T(T)
    np.testing.assert_array_equal(oracle.backmap(sbar, mod, U), s_ml)


@pytest.mark.parametrize("mod,K", [(oracle.BPSK, 6), (oracle.QPSK, 3)])
def test_jed_ml_via_T_equals_complex_ml(mod, K):
    """eq. (4) and eq. (5) have the same maximiser / minimiser (Section II-B)."""
    d = sim.gen_jed(6, K, mod, 40, 0.0, 22)
    s_ml, _ = ml.ml_jed(d["Y"], d["s0"], mod)
    T = oracle.build_T_jed(d["Y"], d["s0"], mod)
    sbar, _ = ml.ml_over_T(T)
    np.testing.assert_array_equal(oracle.backmap(sbar, mod, K), s_ml)


# ---------------------------------------------------------------- P3, P4: preconditioning, step

def test_preconditioned_T_properties():
    """Section III-C: T~ = D^-1 T D^-1 has unit diagonal (minus one for eq. (5),
    reading R3), is symmetric and bounded by one (Cauchy-Schwarz)."""
    H, y, _ = _mimo(32, 8, oracle.QPSK, 30, 10.0, 31)
    D, Tt, deg = oracle.precondition(oracle.build_T_coherent(H, y, oracle.QPSK))
    assert not deg.any()
    np.testing.assert_allclose(np.diagonal(Tt, axis1=1, axis2=2), 1.0, atol=1e-15)
    np.testing.assert_array_equal(Tt, np.swapaxes(Tt, 1, 2))
    assert np.abs(Tt).max() <= 1.0 + 1e-15
    d = sim.gen_jed(16, 16, oracle.QPSK, 10, 5.0, 31)
    Dj, Ttj, _ = oracle.precondition(oracle.build_T_jed(d["Y"], d["s0"], oracle.QPSK))
    np.testing.assert_allclose(np.diagonal(Ttj, axis1=1, axis2=2), -1.0, atol=1e-15)
    assert np.all(Dj > 0)


def test_spectral_norm_matches_svd():
    """||T~||_2 (Section III-B) from eigvalsh equals the largest singular value."""
    H, y, _ = _mimo(32, 8, oracle.QPSK, 30, 10.0, 32)
    _, Tt, _ = oracle.precondition(oracle.build_T_coherent(H, y, oracle.QPSK))
    lam = oracle.spectral_norm(Tt)
    svd = np.array([np.linalg.norm(t, 2) for t in Tt])
    np.testing.assert_allclose(lam, svd, rtol=1e-12)
    d = sim.gen_jed(16, 16, oracle.QPSK, 10, 5.0, 32)
    _, Ttj, _ = oracle.precondition(oracle.build_T_jed(d["Y"], d["s0"], oracle.QPSK))
    np.testing.assert_allclose(oracle.spectral_norm(Ttj), [np.linalg.norm(t, 2) for t in Ttj], rtol=1e-12)


def test_step_size_uses_preconditioned_norm():
    """Algorithm 1 input tau = alpha / ||T~||_2 (not ||T||_2)."""
    H, y, _ = _mimo(32, 8, oracle.QPSK, 10, 10.0, 33)
    r = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.55, t_max=0)
    svd = np.array([np.linalg.norm(t, 2) for t in r["Tt"]])
    np.testing.assert_allclose(r["tau"] * svd, 0.55, rtol=1e-12)


# ---------------------------------------------------------------- P5: first iteration

@pytest.mark.parametrize("mod", [oracle.QPSK, oracle.BPSK])
def test_first_iteration_closed_form_and_matched_filter(mod):
    """Algorithm 1 from L~(0) = D: L~ T~ = T D^-1, so V(1) = D - 2 tau tril(T D^-1),
    and after the positive column scaling the last-row signs are those of
    -T_{N,k}, i.e. the matched filter Re/Im(H^H y) (derived by hand)."""
    H, y, _ = _mimo(16, 4, mod, 25, 2.0, 41)
    T = oracle.build_T_coherent(H, y, mod)
    D, Tt, _ = oracle.precondition(T)
    tau = 0.37 / oracle.spectral_norm(Tt)
    L1, _ = oracle.taser_iterate(Tt, D, tau, 1, pin_last=False)
    V1 = D[:, :, None] * np.eye(T.shape[-1]) - np.tril(2 * tau[:, None, None] * T / D[:, None, :])
    expected = V1 * (D / np.linalg.norm(V1, axis=1))[:, None, :]
    np.testing.assert_allclose(L1, expected, rtol=1e-12, atol=1e-12)
    mf = np.einsum("vbu,vb->vu", np.conj(H.astype(np.complex128)), y.astype(np.complex128))
    mf_bar = _sbar_of(mf, mod)
    sbar, _ = oracle.slice_decisions(L1, D)
    np.testing.assert_array_equal(sbar, np.where(mf_bar >= 0, 1, -1))


@pytest.mark.parametrize("mod", [oracle.QPSK, oracle.BPSK])
def test_first_iteration_margin_closed_form(mod):
    """The margin of slice_decisions is the last row of L = L~ D^-1
    (Section III-C, L~ = L D).  After one iteration from L~(0) = D
    (Algorithm 1), column k of V(1) is D_kk (1 - 2 tau) on the diagonal
    (T~_kk = 1) and -2 tau T_ik / D_kk below it, so, derived by hand from T
    itself,  margin_k = V_Nk / ||V_:,k||
             = -2 tau T_Nk / sqrt(D_kk^4 (1 - 2 tau)^2 + 4 tau^2 sum_{i>k} T_ik^2).
    Dividing by D_NN, or not dividing at all, fails this."""
    H, y, _ = _mimo(12, 3, mod, 40, 0.0, 43)
    T = oracle.build_T_coherent(H, y, mod)
    D, Tt, _ = oracle.precondition(T)
    tau = 0.3 / oracle.spectral_norm(Tt)
    N = T.shape[-1]
    res = oracle.run_taser(T, tau=tau, t_max=1, pin_last=True)
    below = np.tril(T, -1) ** 2                       # T_ik^2 for i > k
    col_tail = below.sum(axis=1)                      # sum over i > k, per column k
    Dk = np.sqrt(np.diagonal(T, axis1=1, axis2=2))
    t = tau[:, None]
    expected = -2 * t * T[:, N - 1, :N - 1] / np.sqrt(
        Dk[:, :N - 1] ** 4 * (1 - 2 * t) ** 2 + 4 * t ** 2 * col_tail[:, :N - 1])
    np.testing.assert_allclose(res["margin"], expected, rtol=1e-12, atol=1e-15)


def test_margin_bounded_by_column_norm():
    """Every column of L~ has norm D_kk after the prox (Section III-C), so
    the last-row entry of L = L~ D^-1 lies in [-1, 1], at any SNR, step
    factor and iteration count; a margin divided by the wrong D leaves it."""
    worst = 0.0
    for seed, (mod, U, snr, alpha, t_max) in enumerate([(oracle.QPSK, 4, -6.0, 0.9, 10),
                                                         (oracle.QPSK, 8, 3.0, 0.5, 20),
                                                         (oracle.BPSK, 6, 10.0, 0.99, 5)]):
        H, y, _ = _mimo(10, U, mod, 200, snr, 300 + seed)
        res = oracle.detect_coherent(H, y, mod, alpha=alpha, t_max=t_max)
        worst = max(worst, float(np.abs(res["margin"]).max()))
        # and at the largest margins the bound is reached only by a column
        # whose whole norm sits in its last entry
        assert np.all(np.abs(res["margin"]) <= 1.0 + 1e-12)
    assert worst > 0.5


def test_last_row_mse_hand_value():
    """The unfolded loss (the mean squared error between the last row of
    L = L~ D^-1 and the transmitted real symbols), on values worked by hand:
    vector 0: L~ last row (1, -2) with D = (2, 4) gives (0.5, -0.5) against
    s = (+1, -1): errors 0.25 and 0.25; vector 1: last row (-3, 0) with
    D = (3, 5) gives (-1, 0) against (+1, +1): errors 4 and 1.  Mean over
    the four entries: 5.5 / 4 = 1.375."""
    import torch
    from oracle.unfolded import last_row_mse
    L = torch.zeros(2, 3, 3, dtype=torch.float64)
    L[0, 2, :2] = torch.tensor([1.0, -2.0])
    L[1, 2, :2] = torch.tensor([-3.0, 0.0])
    L[:, 2, 2] = 7.0                                  # held last entry: not part of the loss
    D = torch.tensor([[2.0, 4.0, 7.0], [3.0, 5.0, 7.0]], dtype=torch.float64)
    s = torch.tensor([[1.0, -1.0], [1.0, 1.0]], dtype=torch.float64)
    assert float(last_row_mse(L, D, s)) == 1.375


# ---------------------------------------------------------------- P6: one user / one slot

@pytest.mark.parametrize("t_max", [1, 2, 5, 20])
def test_single_user_bpsk_is_ml(t_max):
    """U = 1 BPSK: every iterate's decision is sign Re(h^H y), which is ML,
    when 2 tau <= 1 (alpha <= 1/2; lambda >= 1 for a unit-diagonal PSD T~)."""
    H, y, _ = _mimo(8, 1, oracle.BPSK, 200, -3.0, 51)
    res = oracle.detect_coherent(H, y, oracle.BPSK, alpha=0.5, t_max=t_max)
    mf = np.einsum("vb,vb->v", np.conj(H[:, :, 0].astype(np.complex128)), y.astype(np.complex128)).real
    np.testing.assert_array_equal(res["sbar"][:, 0], np.where(mf >= 0, 1, -1))
    s_ml, _ = ml.ml_coherent(H, y, oracle.BPSK)
    np.testing.assert_array_equal(res["s_hat"], s_ml)


@pytest.mark.parametrize("alpha", [0.3, 0.9])
def test_single_slot_jed_is_ml(alpha):
    """K = 1 BPSK joint detection: the decision is sign Re(y1^H y0 s0), the ML
    JED answer, at every iteration and for any step size (T~ has -1 diagonal)."""
    d = sim.gen_jed(8, 1, oracle.BPSK, 200, -3.0, 52)
    res = oracle.detect_jed(d["Y"], d["s0"], oracle.BPSK, alpha=alpha, t_max=7)
    Y = d["Y"].astype(np.complex128)
    corr = np.einsum("vb,vb->v", np.conj(Y[:, 1]), Y[:, 0] * d["s0"].astype(np.complex128)[:, None]).real
    np.testing.assert_array_equal(res["sbar"][:, 0], np.where(corr >= 0, 1, -1))
    s_ml, _ = ml.ml_jed(d["Y"], d["s0"], oracle.BPSK)
    np.testing.assert_array_equal(res["s_hat"], s_ml)


# ---------------------------------------------------------------- P7: invariants + descent

@pytest.mark.parametrize("alpha", [0.25, 0.5])
def test_invariants_and_descent(alpha):
    """Every iterate: strictly upper part zero; column k has norm D_kk
    (Section III-C prox); L~_NN = D_NN (reading R6); objective
    Tr(L~ T~ L~^T) non-increasing when tau <= 1/(2||T~||), i.e. alpha <= 1/2
    (the gradient tril(2 L T) is 2||T||-Lipschitz; Proposition 1)."""
    H, y, _ = _mimo(32, 8, oracle.QPSK, 40, 4.0, 61)
    res = oracle.detect_coherent(H, y, oracle.QPSK, alpha=alpha, t_max=1)
    D, Tt, tau = res["D"], res["Tt"], res["tau"]
    L = D[:, :, None] * np.eye(Tt.shape[-1])
    f_prev = oracle.objective(L, Tt)
    for _ in range(30):
        L, _ = oracle.taser_iterate(Tt, D, tau, 1, L0=L)
        assert np.all(np.triu(L, 1) == 0.0)
        np.testing.assert_allclose(np.linalg.norm(L, axis=1), D, rtol=1e-12)
        np.testing.assert_array_equal(L[:, -1, -1], D[:, -1])
        f = oracle.objective(L, Tt)
        assert np.all(f <= f_prev + 1e-12 * np.abs(f_prev))
        f_prev = f


def test_descent_jed_any_alpha():
    """For the negative semidefinite T~ of eq. (5) the objective decreases for
    any step size (the quadratic term of the expansion is <= 0)."""
    d = sim.gen_jed(16, 8, oracle.QPSK, 30, 2.0, 62)
    res = oracle.detect_jed(d["Y"], d["s0"], oracle.QPSK, alpha=0.95, t_max=25, record=True)
    f = res["trace"]["objective"]
    assert np.all(np.diff(f, axis=0) <= 1e-12 * np.abs(f[:-1]))


# ---------------------------------------------------------------- P8: Table I

def _table1(mod, U, t_max):
    rows = json.load(open(os.path.join(GOLDEN, "table1_complexity.json")))["rows"]
    row = rows["QPSK" if mod == oracle.QPSK else "BPSK"]["per_iteration"]
    return t_max * sum(Fraction(c) * U ** p for c, p in row)


@pytest.mark.parametrize("mod,U,t_max", [(oracle.BPSK, 1, 1), (oracle.BPSK, 4, 3), (oracle.BPSK, 7, 2),
                                         (oracle.QPSK, 1, 1), (oracle.QPSK, 3, 3), (oracle.QPSK, 5, 2)])
def test_multiplication_count_matches_table1(mod, U, t_max):
    """Table I: the real multiplications of t_max TASER iterations."""
    H, y, _ = _mimo(2 * U + 2, U, mod, 1, 5.0, 70 + U)
    res = oracle.detect_coherent(H, y, mod, alpha=0.5, t_max=0)
    _, mults = taser_counted(res["Tt"][0].tolist(), res["D"][0].tolist(), 0.1, t_max)
    assert mults == _table1(mod, U, t_max)


def test_counted_loop_matches_batched_oracle():
    """The scalar, entry-by-entry Algorithm 1 equals the batched oracle."""
    H, y, _ = _mimo(10, 3, oracle.QPSK, 6, 6.0, 75)
    res = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.8, t_max=0)
    for v in range(6):
        tau = float(0.8 / res["lam"][v])
        Lc, _ = taser_counted(res["Tt"][v].tolist(), res["D"][v].tolist(), tau, 9)
        Lb, _ = oracle.taser_iterate(res["Tt"][v], res["D"][v], tau, 9, pin_last=False)
        np.testing.assert_allclose(np.array(Lc), Lb, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- P9, P10: exact symmetries

@pytest.mark.parametrize("k", [-3, 2, 5])
def test_power_of_two_scaling_is_exact(k):
    """(H, y) -> (2^k H, 2^k y): T -> 4^k T and D -> 2^k D exactly, T~ and tau
    unchanged, L~ -> 2^k L~ bit for bit (every later step is homogeneous)."""
    H, y, _ = _mimo(32, 8, oracle.QPSK, 20, 8.0, 81)
    a = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.6, t_max=10)
    sc = 2.0 ** k
    b = oracle.detect_coherent(H.astype(np.complex128) * sc, y.astype(np.complex128) * sc,
                               oracle.QPSK, alpha=0.6, t_max=10)
    np.testing.assert_array_equal(b["Tt"], a["Tt"])
    np.testing.assert_array_equal(b["L"], np.ldexp(a["L"], k))
    np.testing.assert_array_equal(b["sbar"], a["sbar"])


def test_row_sign_gauge():
    """Flipping row i of L~ commutes with the update: tril(S L T) = S tril(L T)
    for S = diag(+-1) and column norms are unchanged."""
    H, y, _ = _mimo(16, 4, oracle.QPSK, 10, 3.0, 82)
    r = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.5, t_max=4)
    N = r["Tt"].shape[-1]
    S = np.ones(N)
    S[3] = -1.0
    a, _ = oracle.taser_iterate(r["Tt"], r["D"], r["tau"], 6, L0=r["L"])
    b, _ = oracle.taser_iterate(r["Tt"], r["D"], r["tau"], 6, L0=S[:, None] * r["L"])
    np.testing.assert_array_equal(b, S[:, None] * a)


# ---------------------------------------------------------------- P11: convergence (Prop. 1)

def test_converges_to_critical_point():
    """Proposition 1: with alpha < 1 the iterates converge to a critical point:
    successive iterates stop moving and the gradient tril(2 L~ T~), projected
    on the tangent space of each column's sphere, vanishes (columns k < N)."""
    H, y, _ = _mimo(8, 2, oracle.QPSK, 6, 10.0, 91)
    r = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.5, t_max=3000)
    L, Tt = r["L"], r["Tt"]
    L2, _ = oracle.taser_iterate(Tt, r["D"], r["tau"], 1, L0=L)
    assert np.max(np.abs(L2 - L)) < 1e-9
    G = np.tril(2.0 * L @ Tt)
    N = Tt.shape[-1]
    for k in range(N - 1):
        u = L[:, :, k] / np.linalg.norm(L[:, :, k], axis=1)[:, None]
        g = G[:, :, k]
        resid = g - u * np.sum(u * g, axis=1)[:, None]
        assert np.max(np.abs(resid)) < 1e-7


# ---------------------------------------------------------------- P12: quality vs ML

def test_ml_objective_lower_bounds_taser():
    """ML minimises s~^T T s~ over the same discrete set TASER rounds into."""
    H, y, _ = _mimo(8, 3, oracle.QPSK, 60, 2.0, 101)
    r = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.5, t_max=10)
    st = np.concatenate([r["sbar"].astype(float), np.ones((60, 1))], axis=1)
    f_taser = np.einsum("vn,vnm,vm->v", st, r["T"], st)
    _, f_ml = ml.ml_coherent(H, y, oracle.QPSK)
    assert np.all(f_ml <= f_taser + 1e-9 * np.abs(f_taser))


def test_noiseless_tall_system_recovers_symbols():
    """Noiseless, B >= 4U: s~ lies in the null space of T and TASER finds it."""
    H, y, s = _mimo(64, 8, oracle.QPSK, 100, 0.0, 102, noiseless=True)
    r = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.5, t_max=10)
    rate = np.mean(np.all(r["s_hat"] == s, axis=1))
    assert rate >= 0.99


# ---------------------------------------------------------------- degenerate inputs (reading R8)

def test_degenerate_and_nonfinite_inputs():
    H, y, _ = _mimo(8, 2, oracle.QPSK, 4, 5.0, 111)
    y = y.copy()
    y[1] = 0.0
    H = H.copy()
    H[2, :, 1] = 0.0
    y[3, 0] = np.nan
    r = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.5, t_max=5)
    assert r["status"][0] == 0
    assert r["status"][1] == oracle.VEC_DEGENERATE
    assert r["status"][2] == oracle.VEC_DEGENERATE
    assert r["status"][3] == oracle.VEC_NONFINITE
    for v in (1, 2, 3):
        assert np.all(r["sbar"][v] == 1) and np.all(r["margin"][v] == 0.0)


def test_zero_norm_column_reset():
    """Orthogonal channel columns, y orthogonal to user 0 and 2 tau = 1 give a
    zero first column of V(1): it is reset to D_11 e_1 (status bit 4)."""
    B, U = 4, 2
    H = np.zeros((1, B, U), dtype=np.complex64)
    H[0, 0, 0] = 1.0
    H[0, 1, 1] = 1.0
    y = np.zeros((1, B), dtype=np.complex64)
    y[0, 1] = 1.0 + 1.0j
    y[0, 2] = 0.5
    r = oracle.detect_coherent(H, y, oracle.QPSK, tau=np.array([0.5]), t_max=1)
    assert r["status"][0] & oracle.VEC_ZERO_NORM
    assert r["L"][0, 0, 0] == r["D"][0, 0] and np.all(r["L"][0, 1:, 0] == 0.0)


# ---------------------------------------------------------------- P13 (forward part): unfolded

def test_unfolded_constant_schedule_equals_plain():
    """With alpha_t = alpha for every t, the unfolded forward is Algorithm 1."""
    torch = pytest.importorskip("torch")
    from oracle.unfolded import unfolded_forward
    H, y, _ = _mimo(16, 4, oracle.QPSK, 8, 6.0, 121)
    r = oracle.detect_coherent(H, y, oracle.QPSK, alpha=0.7, t_max=6)
    L = unfolded_forward(torch.from_numpy(r["Tt"]), torch.from_numpy(r["D"]), torch.from_numpy(r["lam"]),
                         torch.full((6,), 0.7, dtype=torch.float64))
    np.testing.assert_allclose(L.numpy(), r["L"], rtol=1e-13, atol=1e-13)
