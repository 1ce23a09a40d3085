"""taser_run_static (no workspace argument, no allocation) through the C ABI:
two calls in a row, the second with a smaller batch, each equal to what
taser_run gives for the same inputs."""
import ctypes

import numpy as np
import pytest

import sim

pytestmark = pytest.mark.gpu


def _run_static(taser, desc, H, y, s0=None, tau=None):
    import torch
    lib = taser.load()
    lib.taser_run_static.restype = ctypes.c_int
    lib.taser_run_static.argtypes = [ctypes.POINTER(taser.Desc)] + [ctypes.c_void_p] * 9
    V, N = desc.num_vectors, taser.problem_size(desc.U, desc.mod)
    dev = y.device
    out = {"sbar": torch.empty((V, N - 1), dtype=torch.int8, device=dev),
           "margin": torch.empty((V, N - 1), dtype=torch.float32, device=dev),
           "status": torch.empty((V,), dtype=torch.int32, device=dev),
           "L": torch.empty((V, N * (N + 1) // 2), dtype=torch.float32, device=dev)}
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = lib.taser_run_static(ctypes.byref(desc), p(H), p(y), p(s0), p(tau), p(out["sbar"]), p(out["margin"]),
                              p(out["status"]), p(out["L"]),
                              ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    assert st == taser.OK, taser.load().taser_status_string(st)
    return out


def _same(a, b):
    import torch
    torch.cuda.synchronize()
    for k in ("sbar", "margin", "status", "L"):
        assert torch.equal(a[k], b[k]), k


def test_run_static_matches_run_two_calls(gpu_lib):
    """Group path (128x16 QPSK, 16 vectors per channel): the largest batch the
    static state holds, then a smaller one (the second call must not see the
    first call's state), then a per-vector request (no state); each equal
    bit for bit to taser_run."""
    import torch
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    for num_H, snr in ((4096, 6.0), (37, -2.0)):
        d = sim.gen_mimo(128, 16, 2, num_H, 16, snr, sim.seed_for(2, snr_index=70 + num_H % 7))
        H, y = cu(d["H"]), cu(d["y"])
        for prec in (1, 0):
            desc = gpu_lib.make_desc(num_H * 16, 128, 16, 2, prec=prec, y_per_H=16, t_max=10, alpha=0.9)
            ref = gpu_lib.run(desc, H, y, want_margin=True, want_L=True)
            _same(_run_static(gpu_lib, desc, H, y), ref)
    d = sim.gen_jed(16, 16, 2, 300, 4.0, sim.seed_for(5, snr_index=71))
    Y, s0 = cu(d["Y"]), cu(d["s0"])
    desc = gpu_lib.make_desc(300, 16, 16, 2, mode=gpu_lib.JED, prec=1, t_max=20, alpha=0.9)
    _same(_run_static(gpu_lib, desc, None, Y, s0=s0), gpu_lib.run(desc, None, Y, s0, want_margin=True, want_L=True))


def test_run_static_rejects_more_than_its_state_holds(gpu_lib):
    lib = gpu_lib.load()
    lib.taser_run_static.restype = ctypes.c_int
    lib.taser_run_static.argtypes = [ctypes.POINTER(gpu_lib.Desc)] + [ctypes.c_void_p] * 9
    one = ctypes.c_void_p(16)     # never dereferenced: the call fails first
    desc = gpu_lib.make_desc(65536 + 16, 128, 16, 2, y_per_H=16, t_max=10, alpha=0.9)
    assert lib.taser_run_static(ctypes.byref(desc), one, one, None, None, one, None, one, None,
                                None) == gpu_lib.ERR_WORKSPACE
