"""Parity of the per-vector fused kernel (taser_run when vectors do not come
in groups of 16 sharing a channel, and for joint channel estimation and
detection) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
import sim
from parity import assert_L_parity, assert_decisions, unpack_lower

pytestmark = pytest.mark.gpu

PREC_TOL = {1: (2.5 * 2.0 ** -8, 10 * 2.0 ** -8), 2: (4 * 2.0 ** -11, 10 * 2.0 ** -11)}


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_fused(taser, desc, H=None, y=None, s0=None, tau=None):
    import torch
    res = taser.run(desc, None if H is None else _cuda(H), _cuda(y), None if s0 is None else _cuda(s0),
                    tau=None if tau is None else _cuda(tau), want_margin=True, want_L=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


COHERENT = [
    # (B, U, mod, num_H, y_per_H, snr, t_max, alpha)         N  tiles
    (32, 8, oracle.QPSK, 1000, 1, 10.0, 10, 0.5),           # 17 1: the 32x8 parity workload
    (32, 8, oracle.QPSK, 1000, 1, 10.0, 10, 0.9),
    (64, 8, oracle.BPSK, 300, 1, 6.0, 10, 0.5),             # 9  1 (padded)
    (128, 16, oracle.BPSK, 200, 1, 6.0, 10, 0.5),           # 17 1
    (256, 32, oracle.BPSK, 60, 1, 8.0, 10, 0.5),            # 33 2
    (256, 32, oracle.QPSK, 60, 1, 8.0, 10, 0.5),            # 65 4
    (12, 5, oracle.QPSK, 131, 1, 3.0, 7, 0.7),              # 11 1 (ragged)
    (100, 12, oracle.QPSK, 40, 4, 5.0, 10, 0.5),            # 25 2, 4 vectors per channel
    (40, 30, oracle.QPSK, 30, 1, 15.0, 5, 0.6),             # 61 4 (overloaded-ish, padded)
]


@pytest.mark.parametrize("case", COHERENT, ids=lambda c: f"B{c[0]}U{c[1]}m{c[2]}V{c[3]*c[4]}a{c[7]}")
def test_vec_coherent(gpu_lib, case):
    B, U, mod, nH, yph, snr, t_max, alpha = case
    d = sim.gen_mimo(B, U, mod, nH, yph, snr, sim.seed_for(3, shard=B + U + mod))
    V = nH * yph
    ref = oracle.detect_coherent(np.repeat(d["H"], yph, axis=0), d["y"], mod, alpha=alpha, t_max=t_max)
    N = oracle.problem_size(U, mod)
    # tau from the oracle: isolates the kernel from the eigenvalue estimate
    desc = gpu_lib.make_desc(V, B, U, mod, tau_mode=gpu_lib.TAU_GIVEN, y_per_H=yph, t_max=t_max)
    g = run_fused(gpu_lib, desc, d["H"], d["y"], tau=ref["tau"].astype(np.float32))
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])
    np.testing.assert_array_equal(g["status"], ref["status"])
    # tau from the in-kernel Lanczos estimate of the norm
    desc = gpu_lib.make_desc(V, B, U, mod, y_per_H=yph, t_max=t_max, alpha=alpha)
    g = run_fused(gpu_lib, desc, d["H"], d["y"])
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])


# Spectra that need many Lanczos steps: real (BPSK) problems with U near B,
# whose T~ has N distinct eigenvalues, and QPSK at N = 65.  (B, U, mod, snr)
# Also rank-deficient T~ with very few antennas, where the Krylov space of
# T~ e_N closes after B (QPSK) or 2B (BPSK) steps.
HARD_SPECTRA = [(64, 32, oracle.BPSK, 4.0), (32, 32, oracle.BPSK, -4.0), (40, 32, oracle.BPSK, 0.0),
                (128, 32, oracle.QPSK, -4.0), (64, 32, oracle.QPSK, 4.0), (32, 16, oracle.QPSK, -4.0),
                (2, 8, oracle.QPSK, 6.0), (3, 16, oracle.BPSK, 6.0), (1, 4, oracle.QPSK, 10.0),
                (8, 1, oracle.BPSK, 3.0), (4, 1, oracle.QPSK, 3.0)]   # N = 2 and 3: two steps


@pytest.mark.parametrize("B, U, mod, snr", HARD_SPECTRA, ids=lambda x: str(x))
@pytest.mark.parametrize("t_max", [1, 10])
def test_vec_spectral_hard_spectra(gpu_lib, B, U, mod, snr, t_max):
    """The per-vector kernel's own step size where the top eigenvalue of T~
    is slow to emerge (BPSK: 16 + N/4 Lanczos steps, QPSK: 12 + N/8): L~
    within 1e-5 of the oracle's, which takes ||T~||_2 from LAPACK.  After one
    iteration L~ moves with tau to first order, so an eigenvalue a few 1e-5
    short already fails."""
    d = sim.gen_mimo(B, U, mod, 256, 1, snr, sim.seed_for(3, snr_index=int(snr) + 70, shard=B + U + mod))
    ref = oracle.detect_coherent(d["H"], d["y"], mod, alpha=0.5, t_max=t_max)
    desc = gpu_lib.make_desc(256, B, U, mod, t_max=t_max, alpha=0.5)
    g = run_fused(gpu_lib, desc, d["H"], d["y"])
    N = oracle.problem_size(U, mod)
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])


JED = [(oracle.QPSK, 16, 16, 600, 20), (oracle.BPSK, 16, 8, 400, 20), (oracle.QPSK, 16, 3, 200, 5),
       (oracle.BPSK, 8, 32, 100, 12), (oracle.QPSK, 24, 30, 50, 10)]


@pytest.mark.parametrize("mod, snr", [(oracle.QPSK, -10.0), (oracle.QPSK, -4.0), (oracle.QPSK, -2.0),
                                      (oracle.QPSK, 0.0), (oracle.QPSK, 12.0), (oracle.BPSK, -14.0),
                                      (oracle.BPSK, -6.0)])
def test_vec_jed_spectral_low_snr(gpu_lib, mod, snr):
    """Joint detection with the kernel's own step size over the SNR range of
    the 16x16 BER sweeps (down to -10 dB QPSK, -14 dB BPSK): there noise
    dominates T~ and its top eigenvalue emerges as slowly as in coherent
    detection (12 + N/8 Lanczos steps for QPSK, 16 + N/4 for BPSK).  L~
    within 1e-5 of the oracle, which uses LAPACK's ||T~||_2."""
    d = sim.gen_jed(16, 16, mod, 400, snr, sim.seed_for(5, snr_index=int(snr) + 30, shard=mod))
    ref = oracle.detect_jed(d["Y"], d["s0"], mod, alpha=0.5, t_max=20)
    desc = gpu_lib.make_desc(400, 16, 16, mod, mode=gpu_lib.JED, t_max=20, alpha=0.5)
    g = run_fused(gpu_lib, desc, y=d["Y"], s0=d["s0"])
    assert_L_parity(unpack_lower(g["L"], oracle.problem_size(16, mod)), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])


@pytest.mark.parametrize("mod, Bx", [(oracle.BPSK, 4), (oracle.QPSK, 2), (oracle.QPSK, 4)])
@pytest.mark.parametrize("snr", [-4.0, 0.0])
def test_vec_jed_short_blocks(gpu_lib, mod, Bx, snr):
    """Joint detection of blocks of 16 slots on 2 or 4 antennas with the
    kernel's own step size: T~ has rank at most 2B (BPSK) or B complex
    dimensions (QPSK), its top eigenvalue does not stand out, and the Krylov
    space of T~ e_N closes after that many steps.  L~ within 1e-5 of the
    oracle's."""
    d = sim.gen_jed(Bx, 16, mod, 300, snr, sim.seed_for(5, snr_index=int(snr) + 80, shard=Bx + mod))
    ref = oracle.detect_jed(d["Y"], d["s0"], mod, alpha=0.5, t_max=10)
    desc = gpu_lib.make_desc(300, Bx, 16, mod, mode=gpu_lib.JED, t_max=10, alpha=0.5)
    g = run_fused(gpu_lib, desc, y=d["Y"], s0=d["s0"])
    assert_L_parity(unpack_lower(g["L"], oracle.problem_size(16, mod)), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])


@pytest.mark.parametrize("mod,Bx,K,nb,t_max", JED, ids=lambda x: str(x))
def test_vec_jed(gpu_lib, mod, Bx, K, nb, t_max):
    d = sim.gen_jed(Bx, K, mod, nb, 6.0, sim.seed_for(5, shard=K + Bx))
    ref = oracle.detect_jed(d["Y"], d["s0"], mod, alpha=0.5, t_max=t_max)
    N = oracle.problem_size(K, mod)
    desc = gpu_lib.make_desc(nb, Bx, K, mod, mode=gpu_lib.JED, tau_mode=gpu_lib.TAU_GIVEN, t_max=t_max)
    g = run_fused(gpu_lib, desc, y=d["Y"], s0=d["s0"], tau=ref["tau"].astype(np.float32))
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])
    desc = gpu_lib.make_desc(nb, Bx, K, mod, mode=gpu_lib.JED, t_max=t_max, alpha=0.5)
    g = run_fused(gpu_lib, desc, y=d["Y"], s0=d["s0"])
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
def test_vec_jed_16bit(gpu_lib, prec):
    d = sim.gen_jed(16, 16, oracle.QPSK, 512, 4.0, sim.seed_for(5, shard=77 + prec))
    ref = oracle.detect_jed(d["Y"], d["s0"], oracle.QPSK, alpha=0.5, t_max=20)
    desc = gpu_lib.make_desc(512, 16, 16, oracle.QPSK, mode=gpu_lib.JED, prec=prec, tau_mode=gpu_lib.TAU_GIVEN,
                             t_max=20)
    g = run_fused(gpu_lib, desc, y=d["Y"], s0=d["s0"], tau=ref["tau"].astype(np.float32))
    ltol, mtol = PREC_TOL[prec]
    assert_L_parity(unpack_lower(g["L"], 33), ref["L"], tol=ltol)
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"], tol=mtol)


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
@pytest.mark.parametrize("snr", [-4.0, -2.0])
@pytest.mark.parametrize("alpha", [0.5, 0.9])
@pytest.mark.parametrize("kind", ["coherent64x16", "jed16x16"])
def test_vec_16bit_products_low_snr(gpu_lib, prec, snr, alpha, kind):
    """The per-vector kernel with 16-bit products at -4 and -2 dB (own
    channel 64x16 QPSK, t_max = 10; JED 16 antennas x 16 + 1 slots,
    t_max = 20), 2,048 vectors, the oracle's tau: decisions equal wherever
    the oracle's |margin| >= 10 u, L~ within assert_16bit_low_snr's bound."""
    from parity import assert_16bit_low_snr, rel_frobenius
    seed = sim.seed_for(3 if kind == "coherent64x16" else 5, snr_index=400 + int(snr) + int(10 * alpha),
                        shard=prec)
    if kind == "jed16x16":
        d = sim.gen_jed(16, 16, oracle.QPSK, 2048, snr, seed)
        ref = oracle.detect_jed(d["Y"], d["s0"], oracle.QPSK, alpha=alpha, t_max=20)
        desc = gpu_lib.make_desc(2048, 16, 16, oracle.QPSK, mode=gpu_lib.JED, prec=prec,
                                 tau_mode=gpu_lib.TAU_GIVEN, t_max=20)
        g = run_fused(gpu_lib, desc, y=d["Y"], s0=d["s0"], tau=ref["tau"].astype(np.float32))
    else:
        d = sim.gen_mimo(64, 16, oracle.QPSK, 2048, 1, snr, seed)
        ref = oracle.detect_coherent(d["H"], d["y"], oracle.QPSK, alpha=alpha, t_max=10)
        desc = gpu_lib.make_desc(2048, 64, 16, oracle.QPSK, prec=prec, tau_mode=gpu_lib.TAU_GIVEN, t_max=10)
        g = run_fused(gpu_lib, desc, H=d["H"], y=d["y"], tau=ref["tau"].astype(np.float32))
    u = PREC_TOL[prec][1] / 10
    assert_16bit_low_snr(rel_frobenius(unpack_lower(g["L"], 33), ref["L"]), u, alpha)
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"], tol=10 * u)


def _assert_jed_prox_invariants(Lp, Y, s0, tol=2e-5):
    """Properties of every block's final L~ (Section II-B, III-C,
    Algorithm 1): T = -A^T A with A = [Hbar, ybar], so D_kk = sqrt(|T_kk|)
    is the norm of column k of A, i.e. the norm of data slot k's received
    vector (for both coordinates of a QPSK symbol), and D_NN = ||y_0 s_0||;
    after the prox every column of L~ has norm D_kk and L~_NN = D_NN.  The
    references are those definitions in float64, not the oracle."""
    Yc = Y.astype(np.complex128)
    K = Y.shape[1] - 1
    slot = np.linalg.norm(Yc[:, 1:, :], axis=2)                    # [nb, K]
    N = 2 * K + 1
    Dref = np.concatenate([slot, slot], axis=1)                    # [nb, N - 1]
    DN = np.linalg.norm(Yc[:, 0, :], axis=1) * np.abs(s0.astype(np.complex128))
    r, c = np.tril_indices(N)
    worst = 0.0
    for v0 in range(0, Lp.shape[0], 8192):
        v1 = min(v0 + 8192, Lp.shape[0])
        L = np.zeros((v1 - v0, N, N))
        L[:, r, c] = Lp[v0:v1]
        norms = np.linalg.norm(L, axis=1)
        err = np.abs(norms[:, :N - 1] / Dref[v0:v1] - 1.0)
        errN = np.abs(L[:, N - 1, N - 1] / DN[v0:v1] - 1.0)
        worst = max(worst, float(err.max()), float(errN.max()))
    assert worst <= tol, f"column norm / D_kk off by {worst:.3e}"


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16"])
def test_vec_jed_full_batch_bench_configuration(gpu_lib, prec):
    """The benchmark's joint-detection launch: 262,144 blocks, B = 16,
    K = 16 + pilot, t_max = 20, the swept alpha, tau spectral.  Decisions are
    checked against the oracle on 2,048 sampled blocks; a second launch that
    also writes L~ must repeat them, and the prox's column norms are checked
    on every block."""
    import json
    import os
    alpha = float(json.load(open(os.path.join(os.path.dirname(__file__), "golden", "alpha_star.json")))
                  ["workloads"]["jed16x16"]["alpha_star"])
    nb = 262144
    d = sim.gen_jed(16, 16, oracle.QPSK, nb, 4.0, sim.seed_for(5, snr_index=2))
    desc = gpu_lib.make_desc(nb, 16, 16, oracle.QPSK, mode=gpu_lib.JED, prec=prec, t_max=20, alpha=alpha)
    import torch
    res = gpu_lib.run(desc, None, _cuda(d["Y"]), _cuda(d["s0"]))
    torch.cuda.synchronize()
    sb, st = res["sbar"].cpu().numpy(), res["status"].cpu().numpy()
    assert np.all(st == 0)
    idx = np.sort(np.random.default_rng(13).choice(nb, size=2048, replace=False))
    ref = oracle.detect_jed(d["Y"][idx], d["s0"][idx], oracle.QPSK, alpha=alpha, t_max=20)
    mtol = 1e-4 if prec == 0 else PREC_TOL[prec][1]
    assert_decisions(sb[idx], ref["sbar"], ref["margin"], tol=mtol)
    del res
    res = gpu_lib.run(desc, None, _cuda(d["Y"]), _cuda(d["s0"]), want_L=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(res["sbar"].cpu().numpy(), sb)
    _assert_jed_prox_invariants(res["L"].cpu().numpy(), d["Y"], d["s0"])


@pytest.mark.parametrize("mode", ["jed", "coherent"])
def test_vec_graph_replay(gpu_lib, mode):
    """taser_run on the per-vector kernel captured once in a HIP graph: every
    replay, with eager work and synchronisations in between, reproduces the
    eager result bit for bit (JED 16x16 BF16 at t_max = 20; coherent 64x16
    QPSK FP32 with its own channel per vector)."""
    import torch
    if mode == "jed":
        d = sim.gen_jed(16, 16, oracle.QPSK, 512, 4.0, sim.seed_for(5, snr_index=9))
        desc = gpu_lib.make_desc(512, 16, 16, oracle.QPSK, mode=gpu_lib.JED, prec=gpu_lib.PREC_BF16, t_max=20)
        args = (None, _cuda(d["Y"]), _cuda(d["s0"]))
    else:
        d = sim.gen_mimo(64, 16, oracle.QPSK, 512, 1, 6.0, sim.seed_for(3, snr_index=9))
        desc = gpu_lib.make_desc(512, 64, 16, oracle.QPSK, t_max=10)
        args = (_cuda(d["H"]), _cuda(d["y"]), None)
    eager = gpu_lib.run(desc, *args, want_margin=True, want_L=True)
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in eager.items()}
    out = {k: torch.empty_like(v) for k, v in eager.items()}
    gpu_lib.run(desc, *args, want_margin=True, want_L=True, out=out)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gpu_lib.run(desc, *args, want_margin=True, want_L=True, out=out)
    for rep in range(4):
        for v in out.values():
            v.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in eager:
            assert torch.equal(out[k], eager[k]), (mode, rep, k)
    del graph


def test_vec_degenerate_and_flags(gpu_lib):
    B, U, mod = 32, 8, oracle.QPSK
    d = sim.gen_mimo(B, U, mod, 8, 1, 5.0, 8181)
    H, y = d["H"].copy(), d["y"].copy()
    H[1, :, 3] = 0
    y[2] = 0
    y[3, 4] = np.nan
    H[4, 7, 2] = np.inf
    ref = oracle.detect_coherent(H, y, mod, alpha=0.5, t_max=6)
    desc = gpu_lib.make_desc(8, B, U, mod, t_max=6, alpha=0.5)
    g = run_fused(gpu_lib, desc, H, y)
    np.testing.assert_array_equal(g["status"], ref["status"])
    ok = ref["status"] == 0
    assert_L_parity(unpack_lower(g["L"][ok], 17), ref["L"][ok])
    assert np.all(g["sbar"][~ok] == 1) and np.all(g["margin"][~ok] == 0)
    np.testing.assert_allclose(unpack_lower(g["L"][~ok], 17), ref["L"][~ok], rtol=1e-6)
    # literal last column and t_max = 0
    ref2 = oracle.detect_coherent(d["H"], d["y"], mod, alpha=0.95, t_max=5, pin_last=False)
    desc2 = gpu_lib.make_desc(8, B, U, mod, tau_mode=gpu_lib.TAU_GIVEN, t_max=5, flags=gpu_lib.FLAG_LITERAL_LAST)
    g2 = run_fused(gpu_lib, desc2, d["H"], d["y"], tau=ref2["tau"].astype(np.float32))
    assert_L_parity(unpack_lower(g2["L"], 17), ref2["L"])
    np.testing.assert_array_equal(g2["status"], ref2["status"])
    desc0 = gpu_lib.make_desc(8, B, U, mod, t_max=0, alpha=0.5)
    g0 = run_fused(gpu_lib, desc0, d["H"], d["y"])
    assert np.all(g0["sbar"] == 1)


def test_vec_zero_norm_reset(gpu_lib):
    H = np.zeros((1, 4, 2), dtype=np.complex64)
    H[0, 0, 0] = 1.0
    H[0, 1, 1] = 1.0
    y = np.zeros((1, 4), dtype=np.complex64)
    y[0, 1] = 1.0 + 1.0j
    y[0, 2] = 0.5
    ref = oracle.detect_coherent(H, y, oracle.QPSK, tau=np.array([0.5]), t_max=1)
    desc = gpu_lib.make_desc(1, 4, 2, oracle.QPSK, tau_mode=gpu_lib.TAU_GIVEN, t_max=1)
    g = run_fused(gpu_lib, desc, H, y, tau=np.array([0.5], dtype=np.float32))
    assert g["status"][0] & gpu_lib.VEC_ZERO_NORM
    np.testing.assert_allclose(unpack_lower(g["L"], 5)[0], ref["L"][0], atol=1e-6)


@pytest.mark.parametrize("mod, K, nb", [(oracle.QPSK, 16, 400), (oracle.BPSK, 8, 300), (oracle.QPSK, 3, 129)])
def test_jed_channel_estimate(gpu_lib, mod, K, nb):
    """taser_jed_channel: h = Y [s0; s_r] (eq. (4)) from the detected symbols,
    against the oracle's estimate for every block whose decisions equal the
    oracle's (float32 sum of K + 1 complex products: 1e-5 relative)."""
    import torch
    d = sim.gen_jed(16, K, mod, nb, 6.0, sim.seed_for(5, snr_index=40, shard=K))
    ref = oracle.detect_jed(d["Y"], d["s0"], mod, alpha=0.5, t_max=20)
    desc = gpu_lib.make_desc(nb, 16, K, mod, mode=gpu_lib.JED, t_max=20, alpha=0.5)
    Y, s0 = _cuda(d["Y"]), _cuda(d["s0"])
    res = gpu_lib.run(desc, None, Y, s0)
    h = gpu_lib.jed_channel(desc, Y, s0, res["sbar"])
    torch.cuda.synchronize()
    sb, hg = res["sbar"].cpu().numpy(), h.cpu().numpy()
    same = np.all(sb == ref["sbar"], axis=1)
    assert same.mean() >= 0.99
    hr = ref["h_hat"][same]
    scale = np.abs(hr).max(axis=1, keepdims=True)
    assert np.all(np.abs(hg[same] - hr) <= 1e-5 * scale + 1e-6)
