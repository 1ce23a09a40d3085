"""Reference detectors (Section V-A's comparison) through the C ABI against
oracle/reference.py and the exhaustive ML oracle: matched filter, MMSE,
exhaustive ML and K-best, float32 on the GPU against float64."""
import itertools

import numpy as np
import pytest

import oracle
import sim
from oracle import ml, reference

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def _run(taser, kind, d, B, U, mod, K=5, n0=0.0, yph=1):
    import torch
    V = d["y"].shape[0]
    desc = taser.make_desc(V, B, U, mod, y_per_H=yph)
    H = torch.from_numpy(np.ascontiguousarray(d["H"])).cuda()
    y = torch.from_numpy(np.ascontiguousarray(d["y"])).cuda()
    sb, soft = taser.reference_detect(desc, kind, H, y, K=K, n0=n0, want_soft=True)
    torch.cuda.synchronize()
    return sb.cpu().numpy(), soft.cpu().numpy()


def _Hv(d):
    return np.repeat(d["H"], d["y_per_H"], axis=0)


@pytest.mark.parametrize("B, U, mod, yph", [(128, 16, oracle.QPSK, 16), (32, 32, oracle.QPSK, 1),
                                            (64, 24, oracle.BPSK, 1)])
def test_matched_filter(gpu_lib, B, U, mod, yph):
    """Hbar^T ybar: each entry a sum of 2B float32 products, so its error is
    at most about 2B 2^-24 times the sum of |terms| <= ||h_k|| ||y||; signs
    equal wherever the FP64 value is beyond that."""
    d = sim.gen_mimo(B, U, mod, 512 // yph, yph, 4.0, sim.seed_for(1, snr_index=120, shard=B + U))
    sb, x = _run(gpu_lib, gpu_lib.REF_MF, d, B, U, mod, yph=yph)
    Hv = _Hv(d)
    sb64, x64 = reference.matched_filter(Hv, d["y"], mod)
    Hbar, ybar = oracle.real_decomposition_coherent(Hv, d["y"], mod)
    bound = 2 * B * U32 * np.linalg.norm(Hbar, axis=1) * np.linalg.norm(ybar, axis=1)[:, None]
    assert np.all(np.abs(x - x64) <= bound)
    ok = np.abs(x64) > bound
    np.testing.assert_array_equal(sb[ok], sb64[ok])


@pytest.mark.parametrize("B, U, mod, snr", [(128, 16, oracle.QPSK, 6.0), (32, 32, oracle.QPSK, 10.0),
                                            (64, 24, oracle.BPSK, 0.0), (16, 8, oracle.QPSK, -2.0)])
def test_mmse(gpu_lib, B, U, mod, snr):
    """A float32 Cholesky solve of (Hbar^T Hbar + (N0/2) I) x = Hbar^T ybar has
    a relative error of order kappa u (kappa the condition number, u = 2^-24):
    the bound is 64 kappa u ||x||_inf per vector (the factor covers the
    accumulated rounding of forming the matrix and both triangular solves);
    signs equal wherever |x_64| exceeds it."""
    d = sim.gen_mimo(B, U, mod, 400, 1, snr, sim.seed_for(1, snr_index=121, shard=B + U))
    sb, x = _run(gpu_lib, gpu_lib.REF_MMSE, d, B, U, mod, n0=d["N0"])
    sb64, x64 = reference.mmse(d["H"], d["y"], mod, d["N0"])
    Hbar, _ = oracle.real_decomposition_coherent(d["H"], d["y"], mod)
    A = np.swapaxes(Hbar, 1, 2) @ Hbar + (d["N0"] / 2) * np.eye(Hbar.shape[-1])
    kappa = np.linalg.cond(A)
    bound = 64 * kappa * U32 * np.abs(x64).max(axis=1)
    err = np.abs(x - x64).max(axis=1)
    assert np.all(err <= bound), (err / bound).max()
    ok = np.abs(x64) > bound[:, None]
    np.testing.assert_array_equal(sb[ok], sb64[ok])


def _all_costs(H, y, mod):
    """||ybar - Hbar s||^2 of every candidate (brute force, float64)."""
    Hbar, ybar = oracle.real_decomposition_coherent(H, y, mod)
    M = Hbar.shape[-1]
    S = np.array(list(itertools.product([1.0, -1.0], repeat=M)))
    r = ybar[:, None, :] - np.einsum("vbm,cm->vcb", Hbar, S)
    return np.sum(r * r, axis=-1), S


@pytest.mark.parametrize("B, U, mod, snr", [(16, 10, oracle.BPSK, 2.0), (12, 5, oracle.QPSK, 4.0),
                                            (24, 16, oracle.BPSK, 0.0), (8, 3, oracle.QPSK, -2.0)])
def test_exhaustive_ml(gpu_lib, B, U, mod, snr):
    """The GPU's choice is an ML solution of eq. (1) up to float32 rounding:
    its FP64 residual exceeds the minimum by at most 1e-5 relative (the
    objective is accumulated in float32 and recomputed every 256
    candidates), and it is the FP64 minimiser wherever the runner-up is more
    than that behind; the reported residual is the FP64 one within 1e-4."""
    V = 64 if U < 16 else 8
    d = sim.gen_mimo(B, U, mod, V, 1, snr, sim.seed_for(1, snr_index=122, shard=B + U))
    sb, res = _run(gpu_lib, gpu_lib.REF_ML, d, B, U, mod)
    costs, S = _all_costs(d["H"], d["y"], mod)
    order = np.sort(costs, axis=1)
    best, second = order[:, 0], order[:, 1]
    mine = reference.residual(d["H"], d["y"], mod, sb)
    assert np.all(mine <= best * (1 + 1e-5))
    clear = second > best * (1 + 1e-5)
    S_ml = S[np.argmin(costs, axis=1)].astype(np.int8)
    np.testing.assert_array_equal(sb[clear], S_ml[clear])
    np.testing.assert_allclose(res, mine, rtol=1e-4)
    if U <= 10 or mod == oracle.QPSK:
        s_ml, cost = ml.ml_coherent(d["H"], d["y"], mod)          # complex brute force
        np.testing.assert_allclose(best, cost, rtol=1e-12)


@pytest.mark.parametrize("B, U, mod, snr, K", [(64, 32, oracle.QPSK, 6.0, 5), (64, 16, oracle.QPSK, 4.0, 5),
                                               (128, 16, oracle.QPSK, 0.0, 5), (32, 16, oracle.BPSK, 0.0, 5),
                                               (16, 8, oracle.QPSK, 2.0, 16), (16, 8, oracle.QPSK, 2.0, 1),
                                               (32, 32, oracle.QPSK, 10.0, 5)])
def test_kbest(gpu_lib, B, U, mod, snr, K):
    """K-best with float32 partial distances: R and z come from a float32
    Cholesky factorisation of Hbar^T Hbar, so a partial distance carries a
    relative error of order kappa u (kappa the condition number of
    Hbar^T Hbar, u = 2^-24).  Wherever no level had a near-tie between the
    K-th kept and the best dropped candidate (relative gap above
    max(1e-4, 64 kappa u)) the survivors, hence the decisions, equal the
    FP64 oracle's.  For the tall systems (B >= 2U, kappa ~ 3..30) such
    vectors are at least three quarters of the batch; the square 32x32
    system (kappa ~ 6e3) has almost none, so there only the clear vectors
    and the residual are compared.  The reported residual equals the FP64
    residual of the decision within 1e-4."""
    V = 96
    d = sim.gen_mimo(B, U, mod, V, 1, snr, sim.seed_for(1, snr_index=123, shard=B + U + K))
    sb, res = _run(gpu_lib, gpu_lib.REF_KBEST, d, B, U, mod, K=K)
    sb64, _, gap = reference.kbest(d["H"], d["y"], mod, K, return_gap=True)
    Hbar, _ = oracle.real_decomposition_coherent(d["H"], d["y"], mod)
    kappa = np.linalg.cond(np.swapaxes(Hbar, 1, 2) @ Hbar)
    clear = gap > np.maximum(1e-4, 64 * kappa * U32)
    if B >= 2 * U:
        assert clear.mean() >= 0.75
    np.testing.assert_array_equal(sb[clear], sb64[clear])
    mine = reference.residual(d["H"], d["y"], mod, sb)
    np.testing.assert_allclose(res, mine, rtol=1e-4, atol=1e-4 * np.abs(mine).max())


@pytest.mark.parametrize("B, U, mod", [(8, 4, oracle.BPSK), (6, 2, oracle.QPSK), (4, 1, oracle.BPSK)])
def test_kbest_keeping_every_path_is_ml(gpu_lib, B, U, mod):
    """With K >= 2^M no path is ever dropped, so K-best is exhaustive ML:
    M = 4, 4 and 1 real dimensions with K = 16 give the GPU's exhaustive-ML
    decisions wherever the FP64 runner-up is more than 1e-5 behind."""
    V = 128
    d = sim.gen_mimo(B, U, mod, V, 1, 0.0, sim.seed_for(1, snr_index=124, shard=B + U))
    sb_k, res_k = _run(gpu_lib, gpu_lib.REF_KBEST, d, B, U, mod, K=16)
    sb_m, res_m = _run(gpu_lib, gpu_lib.REF_ML, d, B, U, mod)
    costs, S = _all_costs(d["H"], d["y"], mod)
    order = np.sort(costs, axis=1)
    clear = order[:, 1] > order[:, 0] * (1 + 1e-5)
    S_ml = S[np.argmin(costs, axis=1)].astype(np.int8)
    np.testing.assert_array_equal(sb_k[clear], S_ml[clear])
    np.testing.assert_array_equal(sb_m[clear], S_ml[clear])
    np.testing.assert_allclose(res_k, res_m, rtol=1e-4, atol=1e-4 * np.abs(res_m).max())


@pytest.mark.parametrize("kind", ["mf", "mmse", "kbest"])
def test_shared_channel_matches_repeated_channel(gpu_lib, kind):
    """y_per_H = 8 (eight received vectors per channel matrix) gives the same
    outputs, bit for bit, as the same channel repeated per vector."""
    import torch
    B, U, mod, yph = 32, 8, oracle.QPSK, 8
    d = sim.gen_mimo(B, U, mod, 40, yph, 3.0, sim.seed_for(1, snr_index=125))
    k = {"mf": gpu_lib.REF_MF, "mmse": gpu_lib.REF_MMSE, "kbest": gpu_lib.REF_KBEST}[kind]
    sb1, soft1 = _run(gpu_lib, k, d, B, U, mod, K=5, n0=d["N0"], yph=yph)
    rep = dict(d, H=np.ascontiguousarray(np.repeat(d["H"], yph, axis=0)))
    sb2, soft2 = _run(gpu_lib, k, rep, B, U, mod, K=5, n0=d["N0"], yph=1)
    np.testing.assert_array_equal(sb1, sb2)
    np.testing.assert_array_equal(soft1, soft2)


def test_reference_rejects_and_empty(gpu_lib):
    import ctypes
    lib = gpu_lib.load()
    one = ctypes.c_void_p(16)
    d = gpu_lib.make_desc(8, 16, 12, oracle.QPSK)                 # M = 24 > 20 for ML
    assert lib.taser_reference_detect(ctypes.byref(d), gpu_lib.REF_ML, 5, 0.0, one, one, one, None,
                                      None) == gpu_lib.ERR_UNSUPPORTED
    empty = gpu_lib.make_desc(0, 16, 12, oracle.QPSK)
    assert lib.taser_reference_detect(ctypes.byref(empty), gpu_lib.REF_KBEST, 5, 0.0, None, None, None, None,
                                      None) == gpu_lib.OK
