"""Fixed-point mode (Section IV-C) through the C ABI against the integer
oracle (oracle/fixed.py): the words of T^, D and L~ and the decisions must
be identical (integer work: bit for bit), on the GPU's own preprocessing
outputs, for coherent and joint detection, every register bucket of N, the
benchmark's 128x16 size and degenerate inputs."""
import numpy as np
import pytest

import oracle
import sim
from oracle import fixed

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _prep(taser, desc, H, y, s0=None):
    """taser_build_T on the GPU (float32 T~, D, tau, status) as numpy."""
    import torch
    bt = taser.build_T(desc, None if H is None else _cuda(H), _cuda(y), None if s0 is None else _cuda(s0))
    torch.cuda.synchronize()
    return bt


def _fixed(taser, desc, bt):
    import torch
    words = taser.fixed_quantize(desc, bt["Tt"], bt["D"], bt["tau"])
    out = taser.fixed_solve(desc, words["That"], words["D"], bt["status"].clone())
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in {**words, **out}.items()}


def _oracle_words(bt):
    Tt, D, tau = (bt[k].cpu().numpy() for k in ("Tt", "D", "tau"))
    return fixed.fixed_inputs(Tt, D, tau, product_dtype=np.float32)


def _check(taser, desc, bt, t_max):
    N = taser.problem_size(desc.U, desc.mod)
    g = _fixed(taser, desc, bt)
    That, d = _oracle_words(bt)
    # quantisation: the same float32 product rounded the same way
    np.testing.assert_array_equal(g["That"].reshape(That.shape), That)
    np.testing.assert_array_equal(g["D"].reshape(d.shape), d)
    st_in = bt["status"].cpu().numpy()
    skip = (st_in & (oracle.VEC_DEGENERATE | oracle.VEC_NONFINITE)) != 0
    L, st = fixed.fixed_iterate(That, d, t_max, skip=skip)
    r, c = np.tril_indices(N)
    np.testing.assert_array_equal(g["L"], L[:, r, c])
    np.testing.assert_array_equal(g["sbar"], fixed.fixed_decisions(L))
    np.testing.assert_array_equal(g["status"], st_in | st)
    return g, L


CASES = [
    # (mode, B, U, mod, V, snr, t_max, alpha)            N
    ("coh", 32, 8, oracle.QPSK, 300, 10.0, 10, 0.9),    # 17 (32x8 workload)
    ("coh", 128, 16, oracle.QPSK, 256, 4.0, 10, 0.9),   # 33 (headline size)
    ("coh", 16, 2, oracle.BPSK, 200, 0.0, 7, 0.5),      # 3
    ("coh", 64, 24, oracle.QPSK, 64, 8.0, 10, 0.8),     # 49
    ("coh", 96, 63, oracle.BPSK, 32, 12.0, 5, 0.7),     # 64 (largest)
    ("jed", 16, 16, oracle.QPSK, 256, 2.0, 20, 0.99),   # 33 (JED workload)
    ("jed", 16, 8, oracle.BPSK, 128, 6.0, 12, 0.9),     # 9
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}-{'Q' if c[3] == 2 else 'B'}" for c in CASES])
def test_fixed_point_bit_exact(gpu_lib, case):
    mode, B, U, mod, V, snr, t_max, alpha = case
    if mode == "jed":
        d = sim.gen_jed(B, U, mod, V, snr, sim.seed_for(5, snr_index=90, shard=B + U))
        desc = gpu_lib.make_desc(V, B, U, mod, mode=gpu_lib.JED, t_max=t_max, alpha=alpha)
        bt = _prep(gpu_lib, desc, None, d["Y"], d["s0"])
    else:
        d = sim.gen_mimo(B, U, mod, V, 1, snr, sim.seed_for(1, snr_index=90, shard=B + U))
        desc = gpu_lib.make_desc(V, B, U, mod, t_max=t_max, alpha=alpha)
        bt = _prep(gpu_lib, desc, d["H"], d["y"])
    _check(gpu_lib, desc, bt, t_max)


def test_fixed_point_through_taser_solve(gpu_lib):
    """taser_solve with TASER_PREC_FIXED14 quantises in the kernel exactly as
    taser_fixed_quantize does and returns the words' real values; taser_detect
    on them gives the words' decisions."""
    import torch
    B, U, V, t_max = 128, 16, 512, 10
    d = sim.gen_mimo(B, U, oracle.QPSK, 32, 16, 3.0, sim.seed_for(2, snr_index=91))
    desc = gpu_lib.make_desc(V, B, U, oracle.QPSK, y_per_H=16, t_max=t_max, alpha=0.9)
    bt = _prep(gpu_lib, desc, d["H"], d["y"])
    g = _fixed(gpu_lib, desc, bt)
    fdesc = gpu_lib.make_desc(V, B, U, oracle.QPSK, y_per_H=16, t_max=t_max, alpha=0.9,
                              prec=gpu_lib.PREC_FIXED14)
    Lf = gpu_lib.solve(fdesc, bt["Tt"], bt["D"], bt["tau"], bt["status"].clone())
    sb, _ = gpu_lib.detect(fdesc, Lf, bt["D"])
    torch.cuda.synchronize()
    N = 2 * U + 1
    r, c = np.tril_indices(N)
    words = np.zeros((V, N, N))
    words[:, r, c] = g["L"]
    np.testing.assert_array_equal(Lf.cpu().numpy(), fixed.to_real(words)[:, r, c].astype(np.float32))
    np.testing.assert_array_equal(sb.cpu().numpy(), g["sbar"])


def test_fixed_point_full_batch_sampled(gpu_lib):
    """The benchmark's 65,536-vector 128x16 batch (16 vectors per channel):
    2,048 sampled vectors bit for bit against the oracle; on every vector the
    held last word equals D_NN's, and each column's norm is at most D_kk
    within the rounding of its words and equal to it except where the scale
    factor D_jj / ||v_j|| saturated its word (above 4, when a column of V
    nearly cancels; the 11-fraction-bit reading): at most 1e-4 of the
    columns."""
    import torch
    B, U, V = 128, 16, 65536
    d = sim.gen_mimo(B, U, oracle.QPSK, 4096, 16, 6.0, sim.seed_for(2, snr_index=92))
    desc = gpu_lib.make_desc(V, B, U, oracle.QPSK, y_per_H=16, t_max=10, alpha=0.9)
    bt = _prep(gpu_lib, desc, d["H"], d["y"])
    g = _fixed(gpu_lib, desc, bt)
    idx = np.sort(np.random.default_rng(5).choice(V, 2048, replace=False))
    Tt, D, tau = (bt[k].cpu().numpy()[idx] for k in ("Tt", "D", "tau"))
    That, dq = fixed.fixed_inputs(Tt, D, tau, product_dtype=np.float32)
    L, _ = fixed.fixed_iterate(That, dq, 10)
    N = 33
    r, c = np.tril_indices(N)
    np.testing.assert_array_equal(g["L"][idx], L[:, r, c])
    np.testing.assert_array_equal(g["sbar"][idx], fixed.fixed_decisions(L))
    Dq = g["D"].reshape(V, N)
    assert np.all(g["L"][:, -1] == Dq[:, -1])
    Lfull = np.zeros((8192, N, N))
    short, worst = 0, 0.0
    for v0 in range(0, V, 8192):
        Lfull[:] = 0
        Lfull[:, r, c] = g["L"][v0:v0 + 8192]
        nrm = np.linalg.norm(fixed.to_real(Lfull)[:, :, :N - 1], axis=1)
        rel = nrm / (Dq[v0:v0 + 8192, :N - 1] / 256.0)
        worst = max(worst, float(rel.max()))
        short += int(np.count_nonzero(rel < 1 - 3e-3))
    assert worst <= 1 + 3e-3, worst
    assert short <= 1e-4 * V * (N - 1), short
    del torch


def test_fixed_point_degenerate_and_empty(gpu_lib):
    """A zero channel column makes T_kk = 0: the vector runs no iterations and
    keeps L~ = D (its words) with decisions +1; an empty batch is a no-op."""
    B, U, V = 16, 4, 64
    d = sim.gen_mimo(B, U, oracle.QPSK, V, 1, 5.0, sim.seed_for(1, snr_index=93))
    H = d["H"].copy()
    H[3, :, 1] = 0
    desc = gpu_lib.make_desc(V, B, U, oracle.QPSK, t_max=10, alpha=0.7)
    bt = _prep(gpu_lib, desc, H, d["y"])
    g, L = _check(gpu_lib, desc, bt, 10)
    assert g["status"][3] & oracle.VEC_DEGENERATE
    assert np.all(g["sbar"][3] == 1)
    empty = gpu_lib.make_desc(0, B, U, oracle.QPSK, t_max=10, alpha=0.7)
    import ctypes
    lib = gpu_lib.load()
    assert lib.taser_fixed_solve(ctypes.byref(empty), None, None, None, None, None, None) == gpu_lib.OK
