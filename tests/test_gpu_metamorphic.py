"""Scale equivariance on the GPU.  T of eq. (2) and eq. (5) is quadratic in
the received data, so scaling the inputs by a power of two, (H, y) ->
(2^k H, 2^k y), scales T by 4^k and the preconditioner D of Section III-C by
2^k, leaves T~ and tau unchanged, and scales every iterate L~ of
Algorithm 1 (L~ starts at D and the prox renormalises columns to D_kk) by
exactly 2^k.  In binary floating
point a power-of-two factor only shifts exponents, so every rounding in the
path (products, sums, the 16-bit operand packing, square roots and
reciprocals, whose results depend on the mantissa and the exponent's parity)
is the same, and the kernels must reproduce the scaled result bit for bit:
L~ times 2^k, identical margins (L~_Nk / D_kk), decisions and status.  This
pins the whole path against a mistake that breaks the homogeneity (a dropped
or extra D factor, a constant added where a scaled quantity belongs) without
reference to the oracle.  FP16 operands are left out: their subnormal range
starts at 6e-5, where rounding has a fixed absolute step and a scaled input
may round differently; BF16 has float32's exponent range."""
import numpy as np
import pytest

import sim

pytestmark = pytest.mark.gpu

QPSK, BPSK = 2, 1
SCALES = [3, -2]


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(taser, desc, H, y, s0=None):
    import torch
    res = taser.run(desc, None if H is None else _cuda(H), _cuda(y), None if s0 is None else _cuda(s0),
                    want_margin=True, want_L=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def _assert_scaled(base, scaled, k):
    f = np.float32(2.0 ** k)
    np.testing.assert_array_equal(scaled["L"], base["L"] * f)
    np.testing.assert_array_equal(scaled["margin"], base["margin"])
    np.testing.assert_array_equal(scaled["sbar"], base["sbar"])
    np.testing.assert_array_equal(scaled["status"], base["status"])


def _scale(a, k):
    return (a * np.float32(2.0 ** k)).astype(a.dtype)


@pytest.mark.parametrize("k", SCALES)
@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16"])
def test_group_path_is_scale_equivariant(gpu_lib, prec, k):
    """128x16 QPSK, 16 vectors per channel: the group preparation and solve
    kernels of the headline path, spectral step size."""
    d = sim.gen_mimo(128, 16, QPSK, 48, 16, 8.0, sim.seed_for(2, snr_index=61, shard=prec))
    desc = gpu_lib.make_desc(768, 128, 16, QPSK, prec=prec, y_per_H=16, t_max=10, alpha=0.5)
    base = _run(gpu_lib, desc, d["H"], d["y"])
    assert np.all(base["status"] == 0)
    _assert_scaled(base, _run(gpu_lib, desc, _scale(d["H"], k), _scale(d["y"], k)), k)


@pytest.mark.parametrize("k", SCALES)
@pytest.mark.parametrize("B, U, mod, prec", [(32, 8, QPSK, 0), (32, 8, QPSK, 1), (256, 32, QPSK, 0),
                                             (64, 8, BPSK, 1)])
def test_vector_path_is_scale_equivariant(gpu_lib, B, U, mod, prec, k):
    """Own channel per vector: the per-vector kernel (one to four column tiles)."""
    d = sim.gen_mimo(B, U, mod, 200, 1, 10.0, sim.seed_for(1, snr_index=62, shard=B + U + prec))
    desc = gpu_lib.make_desc(200, B, U, mod, prec=prec, t_max=10, alpha=0.5)
    base = _run(gpu_lib, desc, d["H"], d["y"])
    _assert_scaled(base, _run(gpu_lib, desc, _scale(d["H"], k), _scale(d["y"], k)), k)


@pytest.mark.parametrize("k", SCALES)
@pytest.mark.parametrize("prec", [0, 1])
def test_jed_is_scale_equivariant(gpu_lib, prec, k):
    """JED, 16 antennas, K = 16 + pilot, t_max = 20: scaling the received
    block Y scales T = -A^T A by 4^k."""
    d = sim.gen_jed(16, 16, QPSK, 256, 6.0, sim.seed_for(5, snr_index=63, shard=prec))
    desc = gpu_lib.make_desc(256, 16, 16, QPSK, mode=gpu_lib.JED, prec=prec, t_max=20, alpha=0.5)
    base = _run(gpu_lib, desc, None, d["Y"], d["s0"])
    _assert_scaled(base, _run(gpu_lib, desc, None, _scale(d["Y"], k), d["s0"]), k)


@pytest.mark.parametrize("k", SCALES)
def test_staged_path_is_scale_equivariant(gpu_lib, k):
    """build_T -> solve -> detect: T~, D and tau in HBM between the kernels;
    T~ and tau must be bit-identical, D scaled by 2^k."""
    import torch
    d = sim.gen_mimo(64, 16, QPSK, 40, 1, 10.0, sim.seed_for(1, snr_index=64))
    desc = gpu_lib.make_desc(40, 64, 16, QPSK, t_max=10, alpha=0.5)
    out = []
    for H, y in ((d["H"], d["y"]), (_scale(d["H"], k), _scale(d["y"], k))):
        bt = gpu_lib.build_T(desc, _cuda(H), _cuda(y), None, None)
        L = gpu_lib.solve(desc, bt["Tt"], bt["D"], bt["tau"], bt["status"])
        sbar, margin = gpu_lib.detect(desc, L, bt["D"])
        torch.cuda.synchronize()
        r = {n: v.cpu().numpy() for n, v in bt.items()}
        r.update(L=L.cpu().numpy(), sbar=sbar.cpu().numpy(), margin=margin.cpu().numpy())
        out.append(r)
    base, scaled = out
    f = np.float32(2.0 ** k)
    np.testing.assert_array_equal(scaled["Tt"], base["Tt"])
    np.testing.assert_array_equal(scaled["tau"], base["tau"])
    np.testing.assert_array_equal(scaled["D"], base["D"] * f)
    _assert_scaled(base, scaled, k)
