"""Pins of the fixed-point oracle (oracle/fixed.py): Algorithm 1 in the
14-bit arithmetic of Section IV-C, checked against values worked by hand,
exact special cases of the scale unit, saturation, the iteration's
invariants and the floating-point oracle within the quantisation error."""
import json
import os

import numpy as np
import pytest

import oracle
import sim
from oracle import fixed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_one_iteration_worked_by_hand():
    """tests/golden/fixed_point_n2_step.json: one step of an N = 2 problem
    worked by hand, word by word (derivation in the file)."""
    g = json.load(open(os.path.join(GOLDEN, "fixed_point_n2_step.json")))
    T = np.array([g["inputs"]["That"]])
    d = np.array([g["inputs"]["d"]])
    L, st = fixed.fixed_iterate(T, d, g["inputs"]["t_max"])
    np.testing.assert_array_equal(L[0], np.array(g["expected"]["L"]))
    np.testing.assert_array_equal(fixed.fixed_decisions(L)[0], g["expected"]["sbar"])
    lut = fixed.rsqrt_table()
    for i, v in g["expected"]["table"].items():
        assert lut[int(i)] == v, i
    assert st[0] == 0


def test_rsqrt_table_shape():
    """2^11 words of 14 bits with 13 fraction bits (Section IV-C): every used
    entry lies in (1, 2) (as 1/sqrt of (0.5, 2)), strictly decreasing;
    entries below 512 are never indexed."""
    lut = fixed.rsqrt_table()
    assert lut.shape == (2048,)
    used = lut[512:]
    assert np.all(np.diff(used) < 0)
    assert used.min() > 1 << 12 and used.max() < 1 << 14
    assert np.all(lut[:512] == 0)


@pytest.mark.parametrize("q, d, expect", [
    (1 << 16, 256, 2048),     # ||v|| = 1, D = 1: factor 1.0 (2^11)
    (1 << 18, 256, 1024),     # ||v|| = 2, D = 1: factor 0.5
    (1, 1, 2048),             # ||v|| = 2^-8, D = 2^-8: factor 1.0, left-shifted index
    (1 << 14, 256, 4095),     # ||v|| = 1/2, D = 1: 256 * 8190 / 2^9 = 4095.0 (table at index 1024.5)
    (9 << 16, 768, 2047),     # ||v|| = 3, D = 3: bit length 20 (odd shift 9 -> 10), index 576,
                              # table 10918, 768 * 10918 / 2^12 = 2047.1
])
def test_scale_unit_exact_cases(q, d, expect):
    """D_jj / ||v_j|| at powers of two and simple ratios, worked by hand:
    e.g. q = 2^16 has bit length 17, shift 6, index 1024, table 8190
    (2^18 / sqrt(1024.5)), and round(256 * 8190 / 2^10) = round(2047.5)
    = 2048.  Entry i holds the value at i + 1/2, so exact ratios can land
    one unit low."""
    assert int(fixed.scale_factor(np.array([q]), np.array([d]))[0]) == expect


def test_saturation():
    """A V that leaves the 14-bit range is clamped (reading Q1): with
    D_11 = 8191 (31.996) and T^_11 = -2.0, V_11 = D_11 (1 + 2) = 24573 > 8191
    becomes 8191; the column then has norm 8191 (bottom row 0), the scale
    factor is round(8191 * table / 2^(7 + s/2)) for q = 8191^2 and the new
    L~_11 = round(8191 c / 2^11) = 8191 again (clamped)."""
    T = np.array([[[-8192, 0], [0, 0]]])
    d = np.array([[8191, 32]])
    L, _ = fixed.fixed_iterate(T, d, 1)
    assert L[0, 0, 0] == 8191 and L[0, 1, 0] == 0 and L[0, 1, 1] == 32


def test_invariants_and_held_last_entry():
    """Strictly upper part zero, L~_NN equal to its 5-bit register value at
    every iteration count, column norms within the rounding of D_kk."""
    d = sim.gen_mimo(32, 8, oracle.QPSK, 64, 1, 3.0, 9101)
    r = oracle.detect_coherent(d["H"], d["y"], oracle.QPSK, alpha=0.7, t_max=5)
    T, dq = fixed.fixed_inputs(r["Tt"], r["D"], r["tau"])
    for t_max in (0, 1, 7):
        L, st = fixed.fixed_iterate(T, dq, t_max)
        N = L.shape[-1]
        assert np.all(L[:, np.triu_indices(N, 1)[0], np.triu_indices(N, 1)[1]] == 0)
        np.testing.assert_array_equal(L[:, N - 1, N - 1], dq[:, N - 1])
        Lr = fixed.to_real(L)
        if t_max:
            nrm = np.linalg.norm(Lr[:, :, :N - 1], axis=1)
            np.testing.assert_allclose(nrm, dq[:, :N - 1] / 256.0, rtol=2e-3)
        else:
            np.testing.assert_array_equal(np.diagonal(L, axis1=1, axis2=2)[:, :N - 1], dq[:, :N - 1])


@pytest.mark.parametrize("B, U, snr, alpha", [(32, 8, 4.0, 0.5), (128, 16, 6.0, 0.9), (16, 4, 0.0, 0.5)])
def test_tracks_the_floating_point_oracle(B, U, snr, alpha):
    """Quantising the FP64 oracle's T^ and D and iterating in fixed point
    stays within the quantisation error of Algorithm 1: each stored word is
    off by at most 2^-9 (8 fraction bits) on entries of size up to D_kk, so
    ||L~_fixed - L~_64||_F / ||L~_64||_F stays near sqrt(N(N+1)/2) 2^-9 /
    ||L~||_F ~ 1e-3; the bound is 2^-7.  Decisions agree wherever the
    oracle's |margin| >= 2^-4.  A dropped term, a wrong shift or a wrong
    index moves L~ by far more."""
    d = sim.gen_mimo(B, U, oracle.QPSK, 150, 1, snr, 8000 + B + U)
    r = oracle.detect_coherent(d["H"], d["y"], oracle.QPSK, alpha=alpha, t_max=10)
    T, dq = fixed.fixed_inputs(r["Tt"], r["D"], r["tau"])
    L, _ = fixed.fixed_iterate(T, dq, 10)
    Lr = fixed.to_real(L)
    e = np.linalg.norm((Lr - r["L"]).reshape(150, -1), axis=1) / np.linalg.norm(r["L"].reshape(150, -1), axis=1)
    assert e.max() <= 2.0 ** -7, e.max()
    bad = (fixed.fixed_decisions(L) != r["sbar"]) & (np.abs(r["margin"]) >= 2.0 ** -4)
    assert not bad.any()


def test_degenerate_vectors_skip_and_zero_norm_reset():
    """Skipped vectors keep L~ = D (reading Q8); a column whose V is zero is
    reset to D_jj e_j and flagged."""
    T = np.zeros((2, 3, 3), dtype=np.int64)
    T[:, 0, 0] = 4096          # 2 tau T~_11 = 1: V_11 = D_11 (1 - 1) = 0, column 1 of V is zero
    d = np.array([[300, 200, 64], [300, 200, 64]])
    L, st = fixed.fixed_iterate(T, d, 2, skip=np.array([False, True]))
    assert st[0] == fixed.VEC_ZERO_NORM and st[1] == 0
    assert L[0, 0, 0] == 300 and L[0, 1, 0] == 0 and L[0, 2, 0] == 0
    np.testing.assert_array_equal(np.diagonal(L[1]), [300, 200, 64])
