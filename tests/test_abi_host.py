"""Host-only checks of libtaser.so: it loads, exports every declared symbol
and rejects bad arguments synchronously (no device work is started)."""
import ctypes
import os
import re

import pytest

import paper_1609_01797_amd as taser

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "taser.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(taser_[A-Za-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = taser.load()
    names = declared_functions()
    assert "taser_build_T" in names and "taser_solve" in names and "taser_detect" in names
    for name in names:
        assert hasattr(lib, name), name


def test_abi_version_and_sizes():
    lib = taser.load()
    assert lib.taser_abi_version() == 3
    assert lib.taser_problem_size(16, taser.QPSK) == 33
    assert lib.taser_problem_size(32, taser.BPSK) == 33
    assert lib.taser_problem_size(0, taser.QPSK) == -1
    assert lib.taser_problem_size(4, 7) == -1
    assert b"TASER_ERR_SHAPE" in lib.taser_status_string(taser.ERR_SHAPE)


def _d(**kw):
    base = dict(V=64, B=32, U=8, mod=taser.QPSK)
    base.update(kw)
    return taser.make_desc(**base)


@pytest.mark.parametrize("kw,expect", [
    (dict(), taser.OK),
    (dict(mod=3), taser.ERR_ARG),
    (dict(mode=2), taser.ERR_ARG),
    (dict(prec=9), taser.ERR_ARG),
    (dict(prec=3), taser.OK),               # TASER_PREC_FIXED14 (taser_solve only)
    (dict(tau_mode=2), taser.ERR_ARG),
    (dict(flags=2), taser.ERR_ARG),
    (dict(t_max=-1), taser.ERR_ARG),
    (dict(alpha=0.0), taser.ERR_ARG),
    (dict(alpha=1.0), taser.ERR_ARG),
    (dict(alpha=float("nan")), taser.ERR_ARG),
    (dict(alpha=2.0, tau_mode=taser.TAU_GIVEN), taser.OK),
    (dict(V=-1), taser.ERR_SHAPE),
    (dict(V=1 << 30), taser.OK),            # TASER_MAX_VECTORS
    (dict(V=(1 << 30) + 16), taser.ERR_SHAPE),
    (dict(B=0), taser.ERR_SHAPE),
    (dict(U=0), taser.ERR_SHAPE),
    (dict(U=65), taser.ERR_SHAPE),          # N = 131 > TASER_MAX_N
    (dict(U=64), taser.OK),                 # N = 129
    (dict(y_per_H=0), taser.ERR_SHAPE),
    (dict(y_per_H=5), taser.ERR_SHAPE),     # does not divide V
    (dict(y_per_H=16), taser.OK),
    (dict(mode=taser.JED, y_per_H=2), taser.ERR_SHAPE),
])
def test_check_desc(kw, expect):
    assert taser.check_desc(_d(**kw)) == expect


def test_entry_points_reject_before_any_launch():
    lib = taser.load()
    bad = _d(mod=5)
    z = ctypes.c_void_p(0)
    assert lib.taser_build_T(ctypes.byref(bad), z, z, z, z, z, z, z, z, z) == taser.ERR_ARG
    assert lib.taser_solve(ctypes.byref(bad), z, z, z, z, z, z) == taser.ERR_ARG
    assert lib.taser_detect(ctypes.byref(bad), z, z, z, z, z) == taser.ERR_ARG
    assert lib.taser_run(ctypes.byref(bad), z, z, z, z, z, z, z, z, z, 0, z) == taser.ERR_ARG
    good = _d()
    # valid descriptor, null buffers: rejected synchronously
    assert lib.taser_build_T(ctypes.byref(good), z, z, z, z, z, z, z, z, z) == taser.ERR_ARG
    assert lib.taser_solve(ctypes.byref(good), z, z, z, z, z, z) == taser.ERR_ARG
    assert lib.taser_detect(ctypes.byref(good), z, z, z, z, z) == taser.ERR_ARG
    # nothing to do: OK without touching the device
    empty = _d(V=0)
    assert lib.taser_build_T(ctypes.byref(empty), z, z, z, z, z, z, z, z, z) == taser.OK
    assert lib.taser_solve(ctypes.byref(empty), z, z, z, z, z, z) == taser.OK
    assert lib.taser_detect(ctypes.byref(empty), z, z, z, z, z) == taser.OK
    # bf16 products are not offered by the staged solve
    assert lib.taser_solve(ctypes.byref(_d(prec=taser.PREC_BF16)), z, z, z, z, z, z) == taser.ERR_UNSUPPORTED
    # a channel too large for the staged build's LDS copy
    assert lib.taser_build_T(ctypes.byref(_d(B=4096, U=16)), z, z, z, z, z, z, z, z, z) in (taser.ERR_ARG, taser.ERR_UNSUPPORTED)


def test_workspace_size_query():
    lib = taser.load()
    n = ctypes.c_size_t(0)
    d = taser.make_desc(65536, 128, 16, taser.QPSK, y_per_H=16)
    assert lib.taser_workspace_size(ctypes.byref(d), ctypes.byref(n)) == taser.OK
    assert n.value == 4096 * 1088 * 4      # 1,088 floats of state per group of 16 vectors
    assert lib.taser_workspace_size(ctypes.byref(d), None) == taser.ERR_ARG
    other = taser.make_desc(64, 32, 8, taser.QPSK)      # per-vector kernel: no workspace
    assert lib.taser_workspace_size(ctypes.byref(other), ctypes.byref(n)) == taser.OK and n.value == 0
    big = taser.make_desc(4, 64, 40, taser.QPSK)        # N = 81: no fused kernel
    assert lib.taser_workspace_size(ctypes.byref(big), ctypes.byref(n)) == taser.ERR_UNSUPPORTED
    # a run with a missing workspace is rejected before any launch
    z = ctypes.c_void_p(0)
    one = ctypes.c_void_p(16)   # non-null but never dereferenced: the call fails first
    assert lib.taser_run(ctypes.byref(d), one, one, z, z, one, z, one, z, z, 0, z) == taser.ERR_WORKSPACE
    # step-size readout: tau pointer and workspace checked before any launch
    assert lib.taser_run_tau(ctypes.byref(d), one, 4096 * 1088 * 4, z, z) == taser.ERR_ARG
    assert lib.taser_run_tau(ctypes.byref(d), one, 16, one, z) == taser.ERR_WORKSPACE
    assert lib.taser_run_tau(ctypes.byref(d), z, 4096 * 1088 * 4, one, z) == taser.ERR_WORKSPACE
    assert lib.taser_run_tau(ctypes.byref(other), one, 1 << 20, one, z) == taser.ERR_UNSUPPORTED


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    d = _d(V=2, B=4, U=2)
    H = torch.zeros((2, 4, 2), dtype=torch.complex64)
    y = torch.zeros((2, 4), dtype=torch.complex64)
    with pytest.raises(ValueError):
        taser.build_T(d, H, y)


def test_mixed_entry_rejects_bad_arguments():
    lib = taser.load()
    z = ctypes.c_void_p(0)
    d = taser.make_desc(10, 1, 1, taser.QPSK, t_max=10)
    n = ctypes.c_size_t(0)
    assert lib.taser_mixed_workspace_size(ctypes.byref(d), ctypes.byref(n)) == taser.OK
    assert n.value >= 3 * 10 * 4
    big = taser.make_desc((1 << 30) + 1, 1, 1, taser.QPSK, t_max=10)
    assert lib.taser_mixed_workspace_size(ctypes.byref(big), ctypes.byref(n)) == taser.ERR_SHAPE
    jd = taser.make_desc(10, 1, 1, taser.QPSK, mode=taser.JED)
    assert lib.taser_mixed_workspace_size(ctypes.byref(jd), ctypes.byref(n)) == taser.ERR_UNSUPPORTED
    launch = taser.MixedLaunch()
    args = [z] * 7
    assert lib.taser_run_mixed(ctypes.byref(d), *args, z, z, z, 64, z, ctypes.byref(launch), z, 0, z) == taser.ERR_ARG
    one = ctypes.c_void_p(16)
    ok_args = [one] * 7
    assert lib.taser_run_mixed(ctypes.byref(d), *ok_args, z, one, z, 32, one, ctypes.byref(launch), one, 1 << 20, z) == taser.ERR_SHAPE
    assert lib.taser_run_mixed(ctypes.byref(d), *ok_args, z, one, z, 64, one, ctypes.byref(launch), one, 8, z) == taser.ERR_WORKSPACE
    launch.blocks[1] = -3
    assert lib.taser_run_mixed(ctypes.byref(d), *ok_args, z, one, z, 64, one, ctypes.byref(launch), one, 1 << 20, z) == taser.ERR_ARG
    launch.blocks[1] = 0
    launch.waves[2] = 2
    assert lib.taser_run_mixed(ctypes.byref(d), *ok_args, z, one, z, 64, one, ctypes.byref(launch), one, 1 << 20, z) == taser.ERR_ARG
    launch.waves[2] = 1
    launch.single_launch = 3
    assert lib.taser_run_mixed(ctypes.byref(d), *ok_args, z, one, z, 64, one, ctypes.byref(launch), one, 1 << 20, z) == taser.ERR_ARG
    launch.single_launch = 0
    launch.concurrent = -1
    assert lib.taser_run_mixed(ctypes.byref(d), *ok_args, z, one, z, 64, one, ctypes.byref(launch), one, 1 << 20, z) == taser.ERR_ARG


def test_fused_entry_points_accept_an_empty_batch():
    """V = 0 is a valid request with nothing to do: every fused entry point
    returns OK with null buffers and starts no device work."""
    lib = taser.load()
    z = ctypes.c_void_p(0)
    for mode, B, U, yph in ((taser.COHERENT, 128, 16, 16), (taser.COHERENT, 32, 8, 1), (taser.JED, 16, 16, 1)):
        d = taser.make_desc(0, B, U, taser.QPSK, mode=mode, y_per_H=yph, t_max=10)
        assert lib.taser_run(ctypes.byref(d), z, z, z, z, z, z, z, z, z, 0, z) == taser.OK
        assert lib.taser_run_static(ctypes.byref(d), z, z, z, z, z, z, z, z, z) == taser.OK
    head = taser.make_desc(0, 128, 16, taser.QPSK, y_per_H=16, t_max=10)
    assert lib.taser_run_prep(ctypes.byref(head), z, z, z, z, z, z, 0, z) == taser.OK
    assert lib.taser_run_solve(ctypes.byref(head), z, z, z, z, z, 0, z) == taser.OK
    assert lib.taser_run_tau(ctypes.byref(head), z, 0, z, z) == taser.OK
    mixed = taser.make_desc(0, 1, 1, taser.QPSK, t_max=10)
    launch = taser.MixedLaunch()
    assert lib.taser_run_mixed(ctypes.byref(mixed), *([z] * 7), z, z, z, 64, z, ctypes.byref(launch),
                               z, 0, z) == taser.OK


def test_unfolded_sizes_and_rejects():
    """Shape and argument checks of the unfolded entry points run on the
    host before any device call."""
    lib = taser.load()
    U = taser.UnfoldedDesc
    ck, ws = ctypes.c_size_t(0), ctypes.c_size_t(0)

    def sizes(u):
        return lib.taser_unfolded_sizes(ctypes.byref(u), ctypes.byref(ck), ctypes.byref(ws))

    assert sizes(U(10, 33, 20, taser.REAL_F32, 5, 0)) == taser.OK
    assert (ck.value, ws.value) == (10 * 4 * 561, 10 * 20 * 4)
    assert sizes(U(3, 9, 5, taser.REAL_F64, 2, taser.FLAG_LITERAL_LAST)) == taser.OK
    assert (ck.value, ws.value) == (3 * 3 * 45, 3 * 5 * 8)
    assert sizes(U(1, 65, 5, taser.REAL_F32, 1, 0)) == taser.ERR_SHAPE
    assert sizes(U((1 << 30) + 1, 9, 5, taser.REAL_F32, 1, 0)) == taser.ERR_SHAPE
    assert sizes(U(1, 1, 5, taser.REAL_F32, 1, 0)) == taser.ERR_SHAPE
    assert sizes(U(1, 9, 0, taser.REAL_F32, 1, 0)) == taser.ERR_SHAPE
    assert sizes(U(1, 9, 5, taser.REAL_F32, 0, 0)) == taser.ERR_SHAPE
    assert sizes(U(-1, 9, 5, taser.REAL_F32, 1, 0)) == taser.ERR_SHAPE
    assert sizes(U(1, 9, 5, 2, 1, 0)) == taser.ERR_ARG
    assert sizes(U(1, 9, 5, taser.REAL_F32, 1, 4)) == taser.ERR_ARG
    # a segment of 64 FP64 states does not fit in LDS
    assert sizes(U(1, 64, 64, taser.REAL_F64, 64, 0)) == taser.ERR_UNSUPPORTED
    z, one = ctypes.c_void_p(0), ctypes.c_void_p(16)
    u = U(4, 9, 5, taser.REAL_F32, 2, 0)
    assert lib.taser_unfolded_forward(ctypes.byref(u), one, one, one, one, z, one, z) == taser.ERR_ARG
    assert lib.taser_unfolded_backward(ctypes.byref(u), one, one, one, one, one, one, one, one, 8,
                                       z) == taser.ERR_WORKSPACE
    assert lib.taser_unfolded_backward(ctypes.byref(u), one, one, one, one, one, z, one, one, 1 << 20,
                                       z) == taser.ERR_ARG
    empty = U(0, 9, 5, taser.REAL_F32, 2, 0)
    assert lib.taser_unfolded_forward(ctypes.byref(empty), z, z, z, z, z, z, z) == taser.OK


def test_calibrate_rejects_bad_arguments():
    lib = taser.load()
    one = ctypes.c_void_p(16)   # never dereferenced: every call below fails first
    fl = ctypes.c_double(0.0)
    assert lib.taser_calibrate_elements() == 1024 * 256
    assert lib.taser_calibrate(3, 10, one, ctypes.byref(fl), None) == taser.ERR_ARG
    assert lib.taser_calibrate(-1, 10, one, ctypes.byref(fl), None) == taser.ERR_ARG
    assert lib.taser_calibrate(0, 0, one, ctypes.byref(fl), None) == taser.ERR_ARG
    assert lib.taser_calibrate(0, (1 << 16) + 1, one, ctypes.byref(fl), None) == taser.ERR_ARG
    assert lib.taser_calibrate(0, 10, None, ctypes.byref(fl), None) == taser.ERR_ARG
    assert lib.taser_calibrate(0, 10, one, None, None) == taser.ERR_ARG


def test_jed_channel_rejects_bad_arguments():
    lib = taser.load()
    one = ctypes.c_void_p(16)   # never dereferenced: every call below fails first
    coh = taser.make_desc(8, 16, 16, taser.QPSK)
    jed = taser.make_desc(8, 16, 16, taser.QPSK, mode=taser.JED)
    assert lib.taser_jed_channel(ctypes.byref(coh), one, one, one, one, None) == taser.ERR_ARG
    assert lib.taser_jed_channel(ctypes.byref(jed), None, one, one, one, None) == taser.ERR_ARG
    assert lib.taser_jed_channel(ctypes.byref(jed), one, one, one, None, None) == taser.ERR_ARG
    empty = taser.make_desc(0, 16, 16, taser.QPSK, mode=taser.JED)
    assert lib.taser_jed_channel(ctypes.byref(empty), None, None, None, None, None) == taser.OK


def test_device_error_path_through_fault_injection():
    """TASER_ERR_DEVICE: with the host-side injection switch armed, every
    entry point that launches device work returns TASER_ERR_DEVICE after its
    argument checks and before launching (so this runs without a GPU); an
    argument error still takes precedence and leaves the injection armed."""
    lib = taser.load()
    z, one = ctypes.c_void_p(0), ctypes.c_void_p(16)   # never dereferenced
    B_ = ctypes.byref
    grp = taser.make_desc(64, 128, 16, taser.QPSK, y_per_H=16, t_max=10)
    vec = taser.make_desc(64, 32, 8, taser.QPSK, t_max=10)
    jed = taser.make_desc(8, 16, 16, taser.QPSK, mode=taser.JED, t_max=20)
    fx = taser.make_desc(64, 32, 8, taser.QPSK, t_max=10, prec=taser.PREC_FIXED14)
    mixed = taser.make_desc(10, 1, 1, taser.QPSK, t_max=10)
    launch = taser.MixedLaunch()
    fl = ctypes.c_double(0.0)
    u = taser.UnfoldedDesc(4, 9, 5, taser.REAL_F32, 2, 0)
    calls = {
        "taser_build_T": lambda: lib.taser_build_T(B_(vec), one, one, z, one, one, one, one, one, z),
        "taser_solve": lambda: lib.taser_solve(B_(vec), one, one, one, one, one, z),
        "taser_detect": lambda: lib.taser_detect(B_(vec), one, one, one, one, z),
        "taser_jed_channel": lambda: lib.taser_jed_channel(B_(jed), one, one, one, one, z),
        "taser_run (group)": lambda: lib.taser_run(B_(grp), one, one, z, z, one, z, one, z, one, 1 << 20, z),
        "taser_run (per-vector)": lambda: lib.taser_run(B_(vec), one, one, z, z, one, z, one, z, z, 0, z),
        "taser_run_static (group)": lambda: lib.taser_run_static(B_(grp), one, one, z, z, one, z, one, z, z),
        "taser_run_static (per-vector)": lambda: lib.taser_run_static(B_(vec), one, one, z, z, one, z, one, z, z),
        "taser_solve (fixed14)": lambda: lib.taser_solve(B_(fx), one, one, one, one, one, z),
        "taser_fixed_quantize": lambda: lib.taser_fixed_quantize(B_(vec), one, one, one, one, one, z),
        "taser_fixed_solve": lambda: lib.taser_fixed_solve(B_(vec), one, one, one, z, one, z),
        "taser_run_prep": lambda: lib.taser_run_prep(B_(grp), one, one, z, z, one, one, 1 << 20, z),
        "taser_run_solve": lambda: lib.taser_run_solve(B_(grp), one, z, one, z, one, 1 << 20, z),
        "taser_run_tau": lambda: lib.taser_run_tau(B_(grp), one, 1 << 20, one, z),
        "taser_calibrate": lambda: lib.taser_calibrate(0, 10, one, B_(fl), z),
        "taser_run_mixed": lambda: lib.taser_run_mixed(B_(mixed), *([one] * 7), z, one, z, 64, one, B_(launch),
                                                       one, 1 << 20, z),
        "taser_unfolded_forward": lambda: lib.taser_unfolded_forward(B_(u), one, one, one, one, one, one, z),
        "taser_unfolded_backward": lambda: lib.taser_unfolded_backward(B_(u), one, one, one, one, one, one, one,
                                                                       one, 1 << 20, z),
    }
    try:
        for name, call in calls.items():
            taser.inject_device_error(1)
            assert call() == taser.ERR_DEVICE, name
        # argument errors come first and do not consume the injection
        taser.inject_device_error(1)
        bad = taser.make_desc(64, 32, 8, 5)
        assert lib.taser_run(B_(bad), one, one, z, z, one, z, one, z, z, 0, z) == taser.ERR_ARG
        assert lib.taser_calibrate(9, 10, one, B_(fl), z) == taser.ERR_ARG
        assert calls["taser_detect"]() == taser.ERR_DEVICE
        assert lib.taser_debug_inject_device_error(-1) == taser.ERR_ARG
        assert b"TASER_ERR_DEVICE" in lib.taser_status_string(taser.ERR_DEVICE)
        with pytest.raises(taser.TaserError):
            taser.inject_device_error(-2)
    finally:
        taser.inject_device_error(0)


def test_workspace_size_per_vector_descriptors():
    """The per-vector path (own channel, JED, any size with N - 1 <= 64 and
    U <= 32) needs no workspace; the group path needs 1,472 floats per 16
    vectors."""
    lib = taser.load()
    n = ctypes.c_size_t(123)
    for d in (taser.make_desc(100, 64, 16, taser.QPSK), taser.make_desc(64, 128, 16, taser.QPSK, y_per_H=8),
              taser.make_desc(32, 16, 16, taser.QPSK, mode=taser.JED), taser.make_desc(7, 256, 32, taser.QPSK),
              taser.make_desc(9, 64, 8, taser.BPSK)):
        n.value = 123
        assert lib.taser_workspace_size(ctypes.byref(d), ctypes.byref(n)) == taser.OK and n.value == 0
    d = taser.make_desc(48, 40, 16, taser.QPSK, y_per_H=16)
    assert lib.taser_workspace_size(ctypes.byref(d), ctypes.byref(n)) == taser.OK
    assert n.value == 3 * 1088 * 4


def test_fixed_point_entry_points_reject_before_any_launch():
    """Fixed-point mode: N <= 64 only, NULL checks, FIXED14 unsupported by the
    fused and mixed paths, empty batches are no-ops (no device work)."""
    lib = taser.load()
    z, one = ctypes.c_void_p(0), ctypes.c_void_p(16)
    big = taser.make_desc(4, 64, 40, taser.QPSK, t_max=10)           # N = 81
    ok = taser.make_desc(4, 32, 8, taser.QPSK, t_max=10)
    fx = taser.make_desc(64, 128, 16, taser.QPSK, y_per_H=16, t_max=10, prec=taser.PREC_FIXED14)
    n = ctypes.c_size_t(0)
    assert lib.taser_fixed_quantize(ctypes.byref(big), one, one, one, one, one, z) == taser.ERR_UNSUPPORTED
    assert lib.taser_fixed_solve(ctypes.byref(big), one, one, one, z, one, z) == taser.ERR_UNSUPPORTED
    assert lib.taser_fixed_quantize(ctypes.byref(ok), one, z, one, one, one, z) == taser.ERR_ARG
    assert lib.taser_fixed_solve(ctypes.byref(ok), one, one, z, z, one, z) == taser.ERR_ARG
    assert lib.taser_fixed_solve(ctypes.byref(ok), one, one, one, z, z, z) == taser.ERR_ARG
    assert lib.taser_workspace_size(ctypes.byref(fx), ctypes.byref(n)) == taser.ERR_UNSUPPORTED
    assert lib.taser_run(ctypes.byref(fx), one, one, z, z, one, z, one, z, one, 1 << 20, z) == taser.ERR_UNSUPPORTED
    assert lib.taser_mixed_workspace_size(ctypes.byref(fx), ctypes.byref(n)) == taser.ERR_UNSUPPORTED
    bigfx = taser.make_desc(4, 64, 40, taser.QPSK, t_max=10, prec=taser.PREC_FIXED14)
    assert lib.taser_solve(ctypes.byref(bigfx), one, one, one, one, one, z) == taser.ERR_UNSUPPORTED
    bf = taser.make_desc(4, 32, 8, taser.QPSK, t_max=10, prec=taser.PREC_BF16)
    assert lib.taser_solve(ctypes.byref(bf), one, one, one, one, one, z) == taser.ERR_UNSUPPORTED
    empty = taser.make_desc(0, 32, 8, taser.QPSK, t_max=10)
    assert lib.taser_fixed_quantize(ctypes.byref(empty), z, z, z, z, z, z) == taser.OK
    assert lib.taser_fixed_solve(ctypes.byref(empty), z, z, z, z, z, z) == taser.OK


def test_reference_detect_rejects_before_any_launch():
    lib = taser.load()
    z, one = ctypes.c_void_p(0), ctypes.c_void_p(16)
    d = taser.make_desc(8, 16, 8, taser.QPSK)
    call = lambda desc, kind, K=5, n0=0.0, sb=one: lib.taser_reference_detect(  # noqa: E731
        ctypes.byref(desc), kind, K, n0, one, one, sb, None, z)
    assert call(d, 7) == taser.ERR_ARG
    assert call(d, taser.REF_KBEST, K=0) == taser.ERR_ARG
    assert call(d, taser.REF_KBEST, K=17) == taser.ERR_ARG
    assert call(d, taser.REF_MMSE, n0=-1.0) == taser.ERR_ARG
    assert call(d, taser.REF_MMSE, n0=float("inf")) == taser.ERR_ARG
    assert call(d, taser.REF_MF, sb=z) == taser.ERR_ARG
    assert call(taser.make_desc(8, 16, 8, taser.QPSK, mode=taser.JED), taser.REF_MF) == taser.ERR_UNSUPPORTED
    assert call(taser.make_desc(8, 16, 33, taser.QPSK), taser.REF_MF) == taser.ERR_UNSUPPORTED   # M = 66
    assert call(taser.make_desc(8, 16, 11, taser.QPSK), taser.REF_ML) == taser.ERR_UNSUPPORTED   # M = 22
    taser.inject_device_error(1)
    try:
        assert call(d, taser.REF_KBEST) == taser.ERR_DEVICE
    finally:
        taser.inject_device_error(0)


def test_sdr_detect_rejects_before_any_launch():
    lib = taser.load()
    z, one = ctypes.c_void_p(0), ctypes.c_void_p(16)
    call = lambda desc, Tt=one, sb=one: lib.taser_sdr_detect(  # noqa: E731
        ctypes.byref(desc), Tt, None, None, sb, None, None, None, None, z)
    assert call(taser.make_desc(4, 64, 33, taser.QPSK)) == taser.ERR_UNSUPPORTED   # N = 67
    assert call(taser.make_desc(4, 64, 65, taser.BPSK)) == taser.ERR_UNSUPPORTED   # N = 66
    assert call(taser.make_desc(0, 16, 8, taser.QPSK), Tt=z, sb=z) == taser.OK
    assert call(taser.make_desc(2, 16, 8, taser.QPSK), Tt=z) == taser.ERR_ARG
    assert call(taser.make_desc(2, 16, 8, taser.QPSK), sb=z) == taser.ERR_ARG
    assert call(taser.make_desc(2, 16, 0, taser.QPSK)) == taser.ERR_SHAPE           # check_desc
    taser.inject_device_error(1)
    try:
        assert call(taser.make_desc(2, 16, 8, taser.QPSK)) == taser.ERR_DEVICE
    finally:
        taser.inject_device_error(0)
