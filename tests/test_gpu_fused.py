"""Parity of the fused single-launch path (taser_run) against the FP64 oracle,
through the C ABI: a slice of the 128x16 QPSK batched workload, the full
65,536-vector batch in the launch configuration the benchmark times (checked
on a sample the oracle computes), degenerate groups and ragged sizes."""
import numpy as np
import pytest

import oracle
import sim
from parity import assert_L_parity, assert_decisions, unpack_lower

pytestmark = pytest.mark.gpu

B, U, N, YPH = 128, 16, 33, 16


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def fused(taser, desc, H, y, tau=None, want_L=True):
    import torch
    res = taser.run(desc, _cuda(H), _cuda(y), tau=None if tau is None else _cuda(tau),
                    want_margin=True, want_L=want_L)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def _assert_prox_invariants(Lp, H, y, y_per_H, tol=2e-5):
    """Properties of every vector's final L~ that hold at any batch size
    (Section III-C, Algorithm 1): after the prox each column k < N has the
    norm D_kk = sqrt(T_kk), and T_kk is the squared norm of the user's
    channel column (the same for its real and imaginary coordinate); the
    held last column is L~_NN = D_NN = ||y||.  The references are those
    definitions in float64, not the oracle."""
    hn = np.linalg.norm(H.astype(np.complex128), axis=1)          # [num_H, U]
    Dref = np.concatenate([hn, hn], axis=1)                         # [num_H, N - 1]
    yn = np.linalg.norm(y.astype(np.complex128), axis=1)            # [V]
    r, c = np.tril_indices(N)
    worst = 0.0
    for v0 in range(0, Lp.shape[0], 8192):
        v1 = min(v0 + 8192, Lp.shape[0])
        L = np.zeros((v1 - v0, N, N))
        L[:, r, c] = Lp[v0:v1]
        norms = np.linalg.norm(L, axis=1)                           # column norms [n, N]
        D = Dref[np.arange(v0, v1) // y_per_H]
        err = np.abs(norms[:, :N - 1] / D - 1.0)
        errN = np.abs(L[:, N - 1, N - 1] / yn[v0:v1] - 1.0)
        worst = max(worst, float(err.max()), float(errN.max()))
    assert worst <= tol, f"column norm / D_kk off by {worst:.3e}"


def _group_oracle(d, alpha, t_max, tau=None, idx=None, pin_last=True):
    Hv = np.repeat(d["H"], d["y_per_H"], axis=0)
    y = d["y"]
    if idx is not None:
        Hv, y = Hv[idx], y[idx]
    return oracle.detect_coherent(Hv, y, oracle.QPSK, alpha=alpha, t_max=t_max, tau=tau, pin_last=pin_last)


@pytest.mark.parametrize("alpha", [0.5, 0.9])
def test_fused_slice_given_tau(gpu_lib, alpha):
    d = sim.gen_mimo(B, U, oracle.QPSK, 64, YPH, 10.0, sim.seed_for(2, shard=1))
    ref = _group_oracle(d, alpha, 10)
    desc = gpu_lib.make_desc(1024, B, U, oracle.QPSK, tau_mode=gpu_lib.TAU_GIVEN, y_per_H=YPH, t_max=10)
    g = fused(gpu_lib, desc, d["H"], d["y"], tau=ref["tau"].astype(np.float32))
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])
    np.testing.assert_array_equal(g["status"], ref["status"])
    np.testing.assert_allclose(g["margin"], ref["margin"], atol=2e-5)


@pytest.mark.parametrize("snr", [0.0, 10.0, 20.0])
def test_fused_slice_spectral(gpu_lib, snr):
    """tau from the in-kernel Lanczos + Laguerre estimate of ||T~||_2."""
    d = sim.gen_mimo(B, U, oracle.QPSK, 64, YPH, snr, sim.seed_for(2, snr_index=int(snr), shard=2))
    ref = _group_oracle(d, 0.5, 10)
    desc = gpu_lib.make_desc(1024, B, U, oracle.QPSK, y_per_H=YPH, t_max=10, alpha=0.5)
    g = fused(gpu_lib, desc, d["H"], d["y"])
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])


def _alpha_star():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "alpha_star.json")
    return float(json.load(open(path))["workloads"]["coherent128x16"]["alpha_star"])


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp32", "bf16", "fp16"])
def test_fused_full_batch_bench_configuration(gpu_lib, prec):
    """The benchmark's launch: 4,096 channels x 16 vectors, tau spectral,
    t_max = 10, the swept alpha, taser_run_prep + taser_run_solve with a
    workspace, no L output.  Decisions are checked on a random sample of
    2,048 vectors against the oracle; L~ on the same sample from a second
    launch that also writes L~, and the prox's column norms on every
    vector."""
    import torch
    alpha = _alpha_star()
    d = sim.gen_mimo(B, U, oracle.QPSK, 4096, YPH, 10.0, sim.seed_for(2, snr_index=5))
    V = 4096 * YPH
    desc = gpu_lib.make_desc(V, B, U, oracle.QPSK, prec=prec, y_per_H=YPH, t_max=10, alpha=alpha)
    H, y = _cuda(d["H"]), _cuda(d["y"])
    ws = torch.empty(gpu_lib.workspace_size(desc), dtype=torch.uint8, device="cuda")
    out = gpu_lib.run_prep(desc, H, y, ws=ws)
    out = gpu_lib.run_solve(desc, out, ws=ws)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    idx = np.sort(np.random.default_rng(7).choice(V, size=2048, replace=False))
    ref = _group_oracle(d, alpha, 10, idx=idx)
    ltol, mtol = (1e-5, 1e-4) if prec == 0 else PREC_TOL[prec]
    assert_decisions(g["sbar"][idx], ref["sbar"], ref["margin"], tol=mtol)
    assert np.all(g["status"] == 0)
    g2 = fused(gpu_lib, desc, d["H"], d["y"], want_L=True)
    np.testing.assert_array_equal(g2["sbar"], g["sbar"])
    assert_L_parity(unpack_lower(g2["L"][idx], N), ref["L"], tol=ltol)
    _assert_prox_invariants(g2["L"], d["H"], d["y"], YPH)


def test_fused_graph_replay(gpu_lib):
    """taser_run_prep + taser_run_solve captured once in a HIP graph (as the
    benchmark replays them): every replay, with eager work and
    synchronisations in between, reproduces the eager result bit for bit."""
    import torch
    d = sim.gen_mimo(B, U, oracle.QPSK, 256, YPH, 2.0, sim.seed_for(2, snr_index=6))
    V = 256 * YPH
    H, y = _cuda(d["H"]), _cuda(d["y"])
    for prec in (0, 1):
        desc = gpu_lib.make_desc(V, B, U, oracle.QPSK, prec=prec, y_per_H=YPH, t_max=10, alpha=0.9)
        ws = torch.empty(gpu_lib.workspace_size(desc), dtype=torch.uint8, device="cuda")
        eager = gpu_lib.run_solve(desc, gpu_lib.run_prep(desc, H, y, ws=ws), want_margin=True, ws=ws)
        eager = {k: v.clone() for k, v in eager.items()}
        out = {k: torch.empty_like(v) for k, v in eager.items()}
        gpu_lib.run_solve(desc, gpu_lib.run_prep(desc, H, y, out=out, ws=ws), want_margin=True, ws=ws)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            gpu_lib.run_prep(desc, H, y, out=out, ws=ws)
            gpu_lib.run_solve(desc, out, want_margin=True, ws=ws)
        for rep in range(4):
            for v in out.values():
                v.zero_()
            ws.zero_()
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            for k in eager:
                assert torch.equal(out[k], eager[k]), (prec, rep, k)
        del graph


def test_fused_degenerate_groups(gpu_lib):
    d = sim.gen_mimo(B, U, oracle.QPSK, 4, YPH, 5.0, 4242)
    H, y = d["H"].copy(), d["y"].copy()
    H[1, :, 3] = 0            # group 1: zero channel column -> every vector degenerate
    y[2 * 16 + 5] = 0         # group 2, vector 5: y = 0
    y[2 * 16 + 9, 7] = np.nan  # group 2, vector 9: non-finite
    H[3, 10, 2] = np.inf      # group 3: non-finite channel
    d2 = dict(d, H=H, y=y)
    ref = _group_oracle(d2, 0.5, 6)
    desc = gpu_lib.make_desc(64, B, U, oracle.QPSK, y_per_H=YPH, t_max=6, alpha=0.5)
    g = fused(gpu_lib, desc, H, y)
    np.testing.assert_array_equal(g["status"], ref["status"])
    ok = ref["status"] == 0
    assert_L_parity(unpack_lower(g["L"][ok], N), ref["L"][ok])
    bad = ~ok
    assert np.all(g["sbar"][bad] == 1) and np.all(g["margin"][bad] == 0)
    np.testing.assert_allclose(unpack_lower(g["L"][bad], N), ref["L"][bad], rtol=1e-6)


@pytest.mark.parametrize("Bx,t_max,flags", [(30, 10, 0), (7, 3, 0), (128, 0, 0), (64, 8, 1),
                                           (100, 10, 0), (45, 10, 0)])
def test_fused_ragged_and_flags(gpu_lib, Bx, t_max, flags):
    d = sim.gen_mimo(Bx, U, oracle.QPSK, 8, 32, 8.0, 777 + Bx)
    ref = _group_oracle(d, 0.7, t_max, pin_last=not flags)
    desc = gpu_lib.make_desc(256, Bx, U, oracle.QPSK, tau_mode=gpu_lib.TAU_GIVEN, y_per_H=32,
                             t_max=t_max, flags=flags)
    g = fused(gpu_lib, desc, d["H"], d["y"], tau=ref["tau"].astype(np.float32))
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])
    np.testing.assert_array_equal(g["status"], ref["status"])


def test_fused_rejects_unsupported(gpu_lib):
    """Problems beyond the fused kernels (N - 1 > 64, or more than 32 users)
    are refused; the staged calls cover them."""
    import torch
    desc = gpu_lib.make_desc(4, 64, 40, oracle.QPSK, y_per_H=1, t_max=10)
    with pytest.raises(gpu_lib.TaserError):
        gpu_lib.run(desc, torch.zeros((4, 64, 40), dtype=torch.complex64, device="cuda"),
                    torch.zeros((4, 64), dtype=torch.complex64, device="cuda"))


# 16-bit products: operands rounded to BF16 (unit roundoff 2^-8) or FP16
# (2^-11), products accumulated and the prox computed in float32.  Over ten
# iterations the relative error of L~ stays within a few unit roundoffs of the
# operand format; the tolerances are 2.5 u (BF16) and 4 u (FP16).  Decisions may
# differ only where the oracle's margin is within the margin error the
# rounding allows (10 u).
PREC_TOL = {1: (2.5 * 2.0 ** -8, 10 * 2.0 ** -8), 2: (4 * 2.0 ** -11, 10 * 2.0 ** -11)}


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
@pytest.mark.parametrize("snr", [0.0, 4.0, 12.0])
def test_fused_16bit_products(gpu_lib, prec, snr):
    d = sim.gen_mimo(B, U, oracle.QPSK, 64, YPH, snr, sim.seed_for(2, snr_index=int(snr) + 20, shard=prec))
    ref = _group_oracle(d, 0.5, 10)
    desc = gpu_lib.make_desc(1024, B, U, oracle.QPSK, prec=prec, tau_mode=gpu_lib.TAU_GIVEN, y_per_H=YPH,
                             t_max=10)
    g = fused(gpu_lib, desc, d["H"], d["y"], tau=ref["tau"].astype(np.float32))
    ltol, mtol = PREC_TOL[prec]
    assert_L_parity(unpack_lower(g["L"], N), ref["L"], tol=ltol)
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"], tol=mtol)
    np.testing.assert_array_equal(g["status"], ref["status"])


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
@pytest.mark.parametrize("snr", [-4.0, -2.0])
@pytest.mark.parametrize("alpha", [0.5, 0.9])
def test_fused_16bit_products_low_snr(gpu_lib, prec, snr, alpha):
    """The low end of the benchmark's SNR sweep, 4,096 vectors, the oracle's
    tau: decisions equal wherever the oracle's |margin| >= 10 u, and the L~
    error bound of assert_16bit_low_snr (per vector for alpha <= 1/2, on
    quantiles for the benchmark's alpha = 0.9)."""
    from parity import assert_16bit_low_snr, rel_frobenius
    d = sim.gen_mimo(B, U, oracle.QPSK, 256, YPH, snr,
                     sim.seed_for(2, snr_index=400 + int(snr) + int(10 * alpha), shard=prec))
    ref = _group_oracle(d, alpha, 10)
    desc = gpu_lib.make_desc(4096, B, U, oracle.QPSK, prec=prec, tau_mode=gpu_lib.TAU_GIVEN, y_per_H=YPH,
                             t_max=10)
    g = fused(gpu_lib, desc, d["H"], d["y"], tau=ref["tau"].astype(np.float32))
    u = PREC_TOL[prec][1] / 10
    assert_16bit_low_snr(rel_frobenius(unpack_lower(g["L"], N), ref["L"]), u, alpha)
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"], tol=10 * u)
    np.testing.assert_array_equal(g["status"], ref["status"])


def test_fused_prep_then_solve_equals_run(gpu_lib):
    """taser_run_prep + taser_run_solve give exactly what taser_run gives, and
    one prep can feed solves of different product precisions."""
    import torch
    d = sim.gen_mimo(B, U, oracle.QPSK, 32, YPH, 3.0, 4343)
    H, y = _cuda(d["H"]), _cuda(d["y"])
    desc = gpu_lib.make_desc(512, B, U, oracle.QPSK, y_per_H=YPH, t_max=10, alpha=0.5)
    ref = gpu_lib.run(desc, H, y, want_margin=True, want_L=True)
    ws = torch.empty(gpu_lib.workspace_size(desc), dtype=torch.uint8, device="cuda")
    out = gpu_lib.run_prep(desc, H, y, ws=ws)
    out = gpu_lib.run_solve(desc, out, want_margin=True, want_L=True, ws=ws)
    torch.cuda.synchronize()
    for k in ("sbar", "status", "margin", "L"):
        assert torch.equal(out[k], ref[k]), k
    desc16 = gpu_lib.make_desc(512, B, U, oracle.QPSK, prec=gpu_lib.PREC_F16, y_per_H=YPH, t_max=10, alpha=0.5)
    ref16 = gpu_lib.run(desc16, H, y, want_L=True)
    out16 = gpu_lib.run_solve(desc16, {"status": out["status"].clone()}, want_L=True, ws=ws, device=H.device)
    torch.cuda.synchronize()
    assert torch.equal(out16["L"], ref16["L"]) and torch.equal(out16["sbar"], ref16["sbar"])


@pytest.mark.parametrize("snr, below", [(-4.0, 3e-5), (0.0, 1e-5), (10.0, 1e-5), (30.0, 1e-5)])
def test_fused_step_size_pin(gpu_lib, snr, below):
    """The preparation's ||T~||_2 (12 Lanczos steps from [c~; 1] + Laguerre,
    float32) against LAPACK's eigvalsh on the oracle's T~, for every vector of
    256 channel groups: lambda = alpha / tau is at most 1e-5 above the exact
    norm and at most `below` under it.  A Ritz value approaches the top
    eigenvalue from below; at -4 dB twelve steps leave about one vector in
    4,000 some 2e-5 short (a slightly larger tau), from 0 dB up all are within
    1e-6.  With TAU_GIVEN, taser_run_tau returns the tau that was passed in,
    bit for bit."""
    import torch
    G = 256
    d = sim.gen_mimo(B, U, oracle.QPSK, G, YPH, snr, sim.seed_for(2, snr_index=int(snr) + 50))
    H, y = _cuda(d["H"]), _cuda(d["y"])
    alpha = 0.5
    desc = gpu_lib.make_desc(G * YPH, B, U, oracle.QPSK, y_per_H=YPH, t_max=10, alpha=alpha)
    ws = torch.empty(gpu_lib.workspace_size(desc), dtype=torch.uint8, device="cuda")
    gpu_lib.run_prep(desc, H, y, ws=ws)
    tau = gpu_lib.run_tau(desc, ws).cpu().numpy().astype(np.float64)
    Hv = np.repeat(d["H"], YPH, axis=0)
    _, Tt, _ = oracle.precondition(oracle.build_T_coherent(Hv, d["y"], oracle.QPSK))
    lam = oracle.spectral_norm(Tt)
    rel = (alpha / tau - lam) / lam
    assert rel.max() <= 1e-5, (rel.max(), int(rel.argmax()))
    assert rel.min() >= -below, (rel.min(), int(rel.argmin()))
    given = gpu_lib.make_desc(G * YPH, B, U, oracle.QPSK, tau_mode=gpu_lib.TAU_GIVEN, y_per_H=YPH, t_max=10)
    t_in = torch.rand(G * YPH, device="cuda", dtype=torch.float32) + 0.1
    gpu_lib.run_prep(given, H, y, tau=t_in, ws=ws)
    assert torch.equal(gpu_lib.run_tau(given, ws), t_in)


@pytest.mark.parametrize("kind, per_lane", [(0, 64.0), (1, 16 * 8192 / 64), (2, 16 * 2048 / 64)])
def test_calibration_kernels(gpu_lib, kind, per_lane):
    """The calibration kernels run, report the flops of their launch (per
    lane and trip: 32 FMAs; 16 MFMAs of 16x16x16 or 16x16x4 per wave) and
    leave finite values that depend on the work."""
    import torch
    out, fl = gpu_lib.calibrate(kind, 8)
    torch.cuda.synchronize()
    assert fl == pytest.approx(1024 * 256 * 8 * per_lane)
    v = out.cpu().numpy()
    assert np.all(np.isfinite(v)) and np.any(v != 0)


@pytest.mark.parametrize("groups", [1, 5, 13])
def test_fused_group_count_not_multiple_of_workgroup(gpu_lib, groups):
    """Group counts that leave waves of the last preparation workgroup without
    a channel group: those waves still take part in the workgroup barriers of
    the step size (tau spectral) and store nothing; every vector matches the
    oracle."""
    d = sim.gen_mimo(B, U, oracle.QPSK, groups, YPH, 10.0, sim.seed_for(2, snr_index=60, shard=groups))
    ref = _group_oracle(d, 0.5, 10)
    desc = gpu_lib.make_desc(groups * YPH, B, U, oracle.QPSK, y_per_H=YPH, t_max=10, alpha=0.5)
    g = fused(gpu_lib, desc, d["H"], d["y"])
    assert_L_parity(unpack_lower(g["L"], N), ref["L"])
    assert_decisions(g["sbar"], ref["sbar"], ref["margin"])
    np.testing.assert_array_equal(g["status"], ref["status"])
