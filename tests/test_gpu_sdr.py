"""Exact SDR detector (eq. (7), Section II-C) through the C ABI against
oracle/sdr.py.  Both solve the SDP in float64 (the GPU to a relative
duality gap of 1e-9, the oracle to 1e-10); the GPU's input T is float32.

Objective: the GPU's X is primal feasible (unit diagonal, factorable), so
Tr(T X_gpu) lies above the optimum by at most the reported duality gap plus
the float32 perturbation of the input (input_err) and float64 rounding.

Decisions: by the Davis-Kahan theorem (Yu, Wang and Samworth's form) the
leading eigenvectors of X_gpu and of the oracle's X satisfy
sin(theta) <= 2 ||X_gpu - X_64||_2 / (lambda_1 - lambda_2) (eigenvalues of
X_64), so after orientation they differ entrywise by at most sqrt(2)
sin(theta); the kernel's power iteration (X^32, then 64 steps) adds at most
EPS_POWER where lambda_2 / lambda_1 <= 0.95 (0.95^2048 is negligible; the
rest is float64 rounding).  Entries whose oracle magnitude exceeds the sum,
with the orienting last entry beyond it too, must give equal signs."""
import numpy as np
import pytest

import oracle
import sim
from oracle import sdr

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
EPS_POWER = 1e-6
U64 = 2.0 ** -53


def _gpu_sdr(taser, desc, Tt, D=None, status=None):
    import torch
    def dev(x):
        if x is None or isinstance(x, torch.Tensor):
            return x
        return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    t, d = dev(Tt), dev(D)
    out = taser.sdr_detect(desc, t, d, status, want_X=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check_against_oracle(g, T, input_err):
    """g: GPU outputs; T [V, N, N] float64; input_err [V]: a bound on
    |Tr((T_gpu - T) X)| for |X_ij| <= 1.  Returns the fraction of decisions
    compared."""
    V, N, _ = T.shape
    ref = sdr.sdr_detect(T)
    X = g["X"].astype(np.float64)
    compared = 0
    for v in range(V):
        np.testing.assert_array_equal(np.diag(g["X"][v]), 1.0)
        assert np.linalg.eigvalsh(X[v]).min() > -1e-10
        absT = np.abs(T[v]).sum()
        delta = input_err[v] + 64 * N * U64 * absT
        exact = float(np.sum(T[v] * X[v]))
        assert abs(g["objective"][v] - exact) <= delta, v
        assert g["gap"][v] >= -delta
        assert exact - ref["objective"][v] <= g["gap"][v] + 2 * delta, v
        assert exact - ref["objective"][v] >= -2 * delta, v
        # decisions: Davis-Kahan against the oracle, then the kernel's own rounding of X_gpu
        lam = ref["eig"][v]
        E = np.linalg.norm(X[v] - ref["X"][v], 2)
        w = np.linalg.eigvalsh(X[v])[::-1]
        if lam[0] - lam[1] <= 0 or w[1] > 0.95 * w[0]:
            continue
        bound = np.sqrt(2.0) * min(1.0, 2.0 * E / (lam[0] - lam[1])) + EPS_POWER
        u = ref["u"][v]
        if abs(u[-1]) > bound:
            ok = np.abs(u[:-1]) > bound
            np.testing.assert_array_equal(g["sbar"][v][ok], ref["sbar"][v][ok], err_msg=f"vector {v}")
            compared += int(ok.sum())
        sb_own, u_own, _ = sdr.round_leading_eigenvector(X[v])
        if abs(u_own[-1]) > EPS_POWER:
            ok = np.abs(u_own[:-1]) > EPS_POWER
            np.testing.assert_array_equal(g["sbar"][v][ok], sb_own[ok], err_msg=f"vector {v} (own X)")
    return compared / (V * (N - 1))


def test_two_by_two_closed_form(gpu_lib):
    """N = 2 (BPSK, one user), T given directly: the optimum T11 + T22 -
    2|T12| = 2.6 at S = [[1, 1], [1, 1]] (off-diagonal -sign(T12) = +1), so
    the decision is +1."""
    T = np.array([[[3.0, -1.2], [-1.2, 2.0]]])
    desc = gpu_lib.make_desc(1, 4, 1, oracle.BPSK)
    g = _gpu_sdr(gpu_lib, desc, T)
    assert 0 <= g["gap"][0] <= 1e-8
    assert abs(g["objective"][0] - 2.6) <= 1e-6            # -1.2 is not a float32
    np.testing.assert_allclose(g["X"][0], [[1.0, 1.0], [1.0, 1.0]], atol=1e-4)
    assert g["sbar"][0, 0] == 1


@pytest.mark.parametrize("B, U, mod, snr", [(8, 3, oracle.QPSK, 0.0), (12, 5, oracle.QPSK, 4.0),
                                            (16, 8, oracle.QPSK, 4.0), (32, 16, oracle.BPSK, 0.0),
                                            (64, 16, oracle.QPSK, 2.0), (32, 32, oracle.BPSK, 8.0),
                                            (128, 63, oracle.BPSK, 6.0), (32, 32, oracle.QPSK, 10.0),
                                            (128, 64, oracle.BPSK, 6.0)])
def test_sdr_given_T(gpu_lib, B, U, mod, snr):
    """T of eq. (2) from the oracle, rounded once to float32 (an input error
    of at most u sum|T_ij|); sizes from N = 7 to the largest supported,
    N = 65, across the three workgroup shapes (N <= 33 and N <= 64 in one
    wave, N = 65 in two)."""
    V = 24 if U < 32 else 8
    d = sim.gen_mimo(B, U, mod, V, 1, snr, sim.seed_for(1, snr_index=130, shard=B + U))
    T = oracle.build_T_coherent(d["H"], d["y"], mod)
    desc = gpu_lib.make_desc(V, B, U, mod)
    g = _gpu_sdr(gpu_lib, desc, T)
    frac = _check_against_oracle(g, T, U32 * np.abs(T).sum(axis=(1, 2)))
    assert frac >= 0.9
    assert np.all(g["iterations"] < 100)


@pytest.mark.parametrize("mode, B, U, mod, snr", [("coh", 128, 8, oracle.QPSK, -2.0), ("coh", 64, 16, oracle.BPSK, -4.0),
                                                  ("coh", 32, 16, oracle.QPSK, 2.0), ("jed", 16, 16, oracle.QPSK, 2.0),
                                                  ("jed", 16, 8, oracle.BPSK, 0.0)])
def test_sdr_after_build_T(gpu_lib, mode, B, U, mod, snr):
    """End to end on the GPU: taser_build_T, then taser_sdr_detect on
    T = D T~ D.  The float32 Gram (eq. (2) / eq. (5)) perturbs each T_ij by
    at most about 2B u D_i D_j (D_i = sqrt|T_ii|), a factor 8 above."""
    import torch
    V = 32
    if mode == "jed":
        d = sim.gen_jed(B, U, mod, V, snr, sim.seed_for(5, snr_index=131, shard=B + U))
        desc = gpu_lib.make_desc(V, B, U, mod, mode=gpu_lib.JED)
        bt = gpu_lib.build_T(desc, None, torch.from_numpy(d["Y"]).cuda(), torch.from_numpy(d["s0"]).cuda())
        T = oracle.build_T_jed(d["Y"], d["s0"], mod)
    else:
        d = sim.gen_mimo(B, U, mod, V, 1, snr, sim.seed_for(1, snr_index=131, shard=B + U))
        desc = gpu_lib.make_desc(V, B, U, mod)
        bt = gpu_lib.build_T(desc, torch.from_numpy(d["H"]).cuda(), torch.from_numpy(d["y"]).cuda())
        T = oracle.build_T_coherent(d["H"], d["y"], mod)
    assert np.all(bt["status"].cpu().numpy() == 0)
    g = _gpu_sdr(gpu_lib, desc, bt["Tt"], bt["D"], bt["status"])
    Dk = np.sqrt(np.abs(np.diagonal(T, axis1=1, axis2=2)))
    err = 16 * B * U32 * Dk.sum(axis=1) ** 2
    frac = _check_against_oracle(g, T, err)
    assert frac >= 0.9


def test_sdr_skips_flagged_vectors(gpu_lib):
    """status != 0 (as taser_build_T flags degenerate or non-finite
    vectors): the vector is not solved; sbar = +1, X = I, zeros."""
    import torch
    V, B, U, mod = 6, 16, 4, oracle.QPSK
    d = sim.gen_mimo(B, U, mod, V, 1, 3.0, sim.seed_for(1, snr_index=132))
    T = oracle.build_T_coherent(d["H"], d["y"], mod)
    status = torch.tensor([0, 1, 0, 2, 0, 0], dtype=torch.int32).cuda()
    desc = gpu_lib.make_desc(V, B, U, mod)
    g = _gpu_sdr(gpu_lib, desc, T, status=status)
    for v in (1, 3):
        assert np.all(g["sbar"][v] == 1)
        assert g["objective"][v] == 0 and g["gap"][v] == 0 and g["iterations"][v] == 0
        np.testing.assert_array_equal(g["X"][v], np.eye(2 * U + 1))
    solved = [0, 2, 4, 5]
    ref = sdr.sdr_detect(T[solved])
    np.testing.assert_allclose(g["objective"][solved], ref["objective"], rtol=1e-5)

