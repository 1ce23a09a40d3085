"""Parity of the staged HIP path (taser_build_T -> taser_solve -> taser_detect)
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import sim
from parity import assert_L_parity, assert_decisions, unpack_lower

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def staged(taser, desc, H, y, s0=None, tau=None):
    import torch
    bt = taser.build_T(desc, None if H is None else _cuda(H), _cuda(y),
                       None if s0 is None else _cuda(s0), None if tau is None else _cuda(tau))
    L = taser.solve(desc, bt["Tt"], bt["D"], bt["tau"], bt["status"])
    sbar, margin = taser.detect(desc, L, bt["D"])
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in bt.items()}
    out.update(L=L.cpu().numpy(), sbar=sbar.cpu().numpy(), margin=margin.cpu().numpy())
    return out


COHERENT_CASES = [
    # (B, U, mod, num_H, y_per_H, snr, t_max, alpha)      N
    (32, 8, oracle.QPSK, 1000, 1, 10.0, 10, 0.5),        # 17: the 32x8 parity workload
    (32, 8, oracle.QPSK, 1000, 1, 10.0, 10, 0.9),
    (128, 16, oracle.QPSK, 32, 16, 10.0, 10, 0.5),       # 33: slice of the batched workload
    (64, 8, oracle.BPSK, 200, 1, 12.0, 10, 0.5),         # 9
    (256, 32, oracle.QPSK, 24, 1, 12.0, 10, 0.5),        # 65
    (12, 5, oracle.QPSK, 77, 1, 4.0, 7, 0.7),            # 11: ragged sizes
    (40, 64, oracle.BPSK, 9, 1, 20.0, 3, 0.4),           # 65: overloaded BPSK
    (160, 64, oracle.QPSK, 6, 1, 12.0, 10, 0.5),         # 129: the largest N accepted
    (8, 1, oracle.BPSK, 50, 1, 3.0, 6, 0.5),             # 2: the smallest N
]


@pytest.mark.parametrize("case", COHERENT_CASES, ids=lambda c: f"B{c[0]}U{c[1]}m{c[2]}V{c[3]*c[4]}a{c[7]}")
def test_staged_coherent_given_tau(gpu_lib, case):
    B, U, mod, nH, yph, snr, t_max, alpha = case
    d = sim.gen_mimo(B, U, mod, nH, yph, snr, sim.seed_for(1, shard=U))
    V = nH * yph
    Hv = np.repeat(d["H"], yph, axis=0)
    ref = oracle.detect_coherent(Hv, d["y"], mod, alpha=alpha, t_max=t_max)
    desc = gpu_lib.make_desc(V, B, U, mod, tau_mode=gpu_lib.TAU_GIVEN, y_per_H=yph, t_max=t_max, alpha=alpha)
    g = staged(gpu_lib, desc, d["H"], d["y"], tau=ref["tau"].astype(np.float32))
    N = oracle.problem_size(U, mod)
    np.testing.assert_allclose(g["D"], ref["D"], rtol=2e-6)
    np.testing.assert_allclose(g["Tt"], ref["Tt"], rtol=0, atol=2e-6)
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])
    np.testing.assert_array_equal(g["status"], ref["status"])
    np.testing.assert_allclose(g["margin"], ref["margin"], atol=1e-5)


@pytest.mark.parametrize("case", COHERENT_CASES[:5], ids=lambda c: f"B{c[0]}U{c[1]}m{c[2]}")
def test_staged_coherent_spectral_tau(gpu_lib, case):
    """tau = alpha/||T~||_2 computed on the GPU (Lanczos) vs LAPACK."""
    B, U, mod, nH, yph, snr, t_max, alpha = case
    d = sim.gen_mimo(B, U, mod, nH, yph, snr, sim.seed_for(1, shard=100 + U))
    V = nH * yph
    ref = oracle.detect_coherent(np.repeat(d["H"], yph, axis=0), d["y"], mod, alpha=alpha, t_max=t_max)
    desc = gpu_lib.make_desc(V, B, U, mod, y_per_H=yph, t_max=t_max, alpha=alpha)
    g = staged(gpu_lib, desc, d["H"], d["y"])
    np.testing.assert_allclose(g["lam"], ref["lam"], rtol=1e-5)
    np.testing.assert_allclose(g["tau"], ref["tau"], rtol=1e-5)
    N = oracle.problem_size(U, mod)
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])


@pytest.mark.parametrize("B, U, mod, snr", [(128, 16, oracle.QPSK, -4.0), (64, 16, oracle.QPSK, 4.0),
                                            (40, 64, oracle.BPSK, 20.0), (40, 64, oracle.BPSK, 0.0),
                                            (16, 32, oracle.QPSK, 10.0), (160, 64, oracle.QPSK, 8.0),
                                            (96, 64, oracle.QPSK, 0.0), (8, 1, oracle.BPSK, 3.0),
                                            (64, 32, oracle.BPSK, 4.0), (128, 64, oracle.BPSK, -4.0),
                                            (80, 64, oracle.BPSK, 0.0), (90, 128, oracle.BPSK, 4.0),
                                            (64, 128, oracle.BPSK, -4.0)])
def test_staged_lambda_pin(gpu_lib, B, U, mod, snr):
    """||T~||_2 of the staged build (Lanczos from the last column of T~ with
    full reorthogonalisation, 12 + N/8 steps for QPSK and 16 + N/4 for BPSK)
    against LAPACK's eigvalsh, 1e-5 relative, at low SNR, for overloaded
    channels, for real problems with U near B (N distinct eigenvalues) and
    at the largest N."""
    d = sim.gen_mimo(B, U, mod, 256, 1, snr, sim.seed_for(1, snr_index=int(snr) + 20, shard=U))
    T = oracle.build_T_coherent(d["H"], d["y"], mod)
    _, Tt, _ = oracle.precondition(T)
    lam = oracle.spectral_norm(Tt)
    desc = gpu_lib.make_desc(256, B, U, mod, t_max=1, alpha=0.5)
    g = staged(gpu_lib, desc, d["H"], d["y"])
    np.testing.assert_allclose(g["lam"], lam, rtol=1e-5)


@pytest.mark.parametrize("mod,K,nb,t_max", [(oracle.QPSK, 16, 512, 20), (oracle.BPSK, 8, 300, 20),
                                            (oracle.QPSK, 3, 100, 5)])
def test_staged_jed(gpu_lib, mod, K, nb, t_max):
    d = sim.gen_jed(16, K, mod, nb, 6.0, sim.seed_for(5, shard=K))
    ref = oracle.detect_jed(d["Y"], d["s0"], mod, alpha=0.5, t_max=t_max)
    desc = gpu_lib.make_desc(nb, 16, K, mod, mode=gpu_lib.JED, tau_mode=gpu_lib.TAU_GIVEN, t_max=t_max)
    g = staged(gpu_lib, desc, None, d["Y"], s0=d["s0"], tau=ref["tau"].astype(np.float32))
    N = oracle.problem_size(K, mod)
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])
    # spectral step on the GPU too
    desc2 = gpu_lib.make_desc(nb, 16, K, mod, mode=gpu_lib.JED, t_max=t_max, alpha=0.5)
    g2 = staged(gpu_lib, desc2, None, d["Y"], s0=d["s0"])
    np.testing.assert_allclose(g2["lam"], ref["lam"], rtol=1e-5)


def test_staged_literal_last_column(gpu_lib):
    B, U, mod = 16, 4, oracle.QPSK
    d = sim.gen_mimo(B, U, mod, 300, 1, -2.0, 77)
    ref = oracle.detect_coherent(d["H"], d["y"], mod, alpha=0.95, t_max=6, pin_last=False)
    desc = gpu_lib.make_desc(300, B, U, mod, tau_mode=gpu_lib.TAU_GIVEN, t_max=6,
                             flags=gpu_lib.FLAG_LITERAL_LAST)
    g = staged(gpu_lib, desc, d["H"], d["y"], tau=ref["tau"].astype(np.float32))
    assert_L_parity(unpack_lower(g["L"], 9), ref["L"])
    np.testing.assert_array_equal(g["status"], ref["status"])


def test_staged_degenerate_and_zero_iterations(gpu_lib):
    B, U, mod = 8, 2, oracle.QPSK
    d = sim.gen_mimo(B, U, mod, 6, 1, 5.0, 78)
    H, y = d["H"].copy(), d["y"].copy()
    y[1] = 0
    H[2, :, 1] = 0
    y[3, 0] = np.nan
    H[4, 0, 0] = np.inf
    ref = oracle.detect_coherent(H, y, mod, alpha=0.5, t_max=5)
    desc = gpu_lib.make_desc(6, B, U, mod, t_max=5, alpha=0.5)
    g = staged(gpu_lib, desc, H, y)
    np.testing.assert_array_equal(g["status"], ref["status"])
    for v in (1, 2, 3, 4):
        assert np.all(g["sbar"][v] == 1) and np.all(g["margin"][v] == 0)
        np.testing.assert_allclose(unpack_lower(g["L"][v:v + 1], 5)[0], ref["L"][v], rtol=1e-6)
    # t_max = 0: L~ = D, every decision +1
    desc0 = gpu_lib.make_desc(6, B, U, mod, t_max=0, alpha=0.5)
    g0 = staged(gpu_lib, desc0, d["H"], d["y"])
    assert np.all(g0["sbar"] == 1)
    L0 = unpack_lower(g0["L"], 5)
    np.testing.assert_allclose(L0, g0["D"][:, :, None] * np.eye(5), rtol=0, atol=0)


def test_staged_zero_norm_reset(gpu_lib):
    H = np.zeros((1, 4, 2), dtype=np.complex64)
    H[0, 0, 0] = 1.0
    H[0, 1, 1] = 1.0
    y = np.zeros((1, 4), dtype=np.complex64)
    y[0, 1] = 1.0 + 1.0j
    y[0, 2] = 0.5
    ref = oracle.detect_coherent(H, y, oracle.QPSK, tau=np.array([0.5]), t_max=1)
    desc = gpu_lib.make_desc(1, 4, 2, oracle.QPSK, tau_mode=gpu_lib.TAU_GIVEN, t_max=1)
    g = staged(gpu_lib, desc, H, y, tau=np.array([0.5], dtype=np.float32))
    assert g["status"][0] & gpu_lib.VEC_ZERO_NORM
    np.testing.assert_allclose(unpack_lower(g["L"], 5)[0], ref["L"][0], atol=1e-6)
