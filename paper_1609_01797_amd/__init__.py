"""Batched TASER detection on AMD MI355X: thin Python binding of libtaser.so.

TASER (Castaneda, Goldstein and Studer, arXiv:1609.01797) is a near-ML
BPSK/QPSK detector for large MU-MIMO systems and a joint channel-estimation
and detection method for SIMO systems.  All arithmetic runs in the HIP
kernels of ``libtaser.so``; this module only checks tensor shapes, dtypes and
devices, allocates outputs with torch (device memory and streams are torch's
job here), and calls the C ABI declared in ``include/taser.h`` on torch's
current stream.  If the library is missing every call raises: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["TaserError", "load", "problem_size", "build_T", "solve", "detect", "run",
           "BPSK", "QPSK", "COHERENT", "JED", "PREC_F32", "PREC_BF16", "PREC_F16", "PREC_FIXED14",
           "REF_MF", "REF_MMSE", "REF_ML", "REF_KBEST", "reference_detect", "sdr_detect",
           "TAU_SPECTRAL", "TAU_GIVEN", "workspace_size", "run_prep", "run_solve", "run_tau", "calibrate", "jed_channel", "run_mixed", "FLAG_LITERAL_LAST", "VEC_DEGENERATE",
           "VEC_NONFINITE", "VEC_ZERO_NORM", "VEC_VNN_NONPOS", "LIB_PATH", "UnfoldedDesc",
           "unfolded_sizes", "unfolded_forward", "unfolded_backward"]

LIB_PATH = os.environ.get("TASER_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                      "libtaser.so")

BPSK, QPSK = 1, 2
COHERENT, JED = 0, 1
PREC_F32, PREC_BF16, PREC_F16, PREC_FIXED14 = 0, 1, 2, 3
TAU_SPECTRAL, TAU_GIVEN = 0, 1
ABI_VERSION = 3           # TASER_ABI_VERSION of include/taser.h (struct layouts of this binding)
FLAG_LITERAL_LAST = 1
VEC_DEGENERATE, VEC_NONFINITE, VEC_ZERO_NORM, VEC_VNN_NONPOS, VEC_UNSUPPORTED = 1, 2, 4, 8, 16

OK, ERR_ARG, ERR_SHAPE, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_DEVICE = 0, -1, -2, -3, -4, -5


class TaserError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("num_vectors", ctypes.c_int32), ("B", ctypes.c_int32), ("U", ctypes.c_int32),
                ("mod", ctypes.c_int32), ("mode", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("tau_mode", ctypes.c_int32), ("y_per_H", ctypes.c_int32),
                ("t_max", ctypes.c_int32), ("flags", ctypes.c_int32), ("alpha", ctypes.c_float)]


class MixedLaunch(ctypes.Structure):
    """Launch choices of a mixed batch (taser_mixed_launch_t): grid per size
    bucket (N-1 <= 16, <= 32, <= 64; 0 = one workgroup per vector, n > 0 = a
    persistent grid of n workgroups), register budget per bucket (0 default,
    1 alternative), single_launch (every bucket in one launch) and
    concurrent (the bucket kernels on three streams)."""
    _fields_ = [("blocks", ctypes.c_int32 * 3), ("waves", ctypes.c_int32 * 3), ("single_launch", ctypes.c_int32),
                ("concurrent", ctypes.c_int32)]


class UnfoldedDesc(ctypes.Structure):
    _fields_ = [("num_vectors", ctypes.c_int32), ("N", ctypes.c_int32), ("t_max", ctypes.c_int32),
                ("real", ctypes.c_int32), ("ckpt_every", ctypes.c_int32), ("flags", ctypes.c_int32)]


REAL_F32, REAL_F64 = 0, 1

_lib = None
_P = ctypes.c_void_p


def load():
    """Load libtaser.so (built by ``python -m paper_1609_01797_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1609_01797_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    D = ctypes.POINTER(Desc)
    lib.taser_abi_version.restype = ctypes.c_int
    if lib.taser_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {lib.taser_abi_version()}, the binding expects "
                          f"{ABI_VERSION}: rebuild it with `python -m paper_1609_01797_amd.build`")
    lib.taser_debug_inject_device_error.restype = ctypes.c_int
    lib.taser_debug_inject_device_error.argtypes = [ctypes.c_int32]
    lib.taser_status_string.restype = ctypes.c_char_p
    lib.taser_status_string.argtypes = [ctypes.c_int]
    lib.taser_problem_size.restype = ctypes.c_int
    lib.taser_problem_size.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.taser_check_desc.restype = ctypes.c_int
    lib.taser_check_desc.argtypes = [D]
    lib.taser_build_T.restype = ctypes.c_int
    lib.taser_build_T.argtypes = [D, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.taser_solve.restype = ctypes.c_int
    lib.taser_solve.argtypes = [D, _P, _P, _P, _P, _P, _P]
    lib.taser_detect.restype = ctypes.c_int
    lib.taser_detect.argtypes = [D, _P, _P, _P, _P, _P]
    lib.taser_workspace_size.restype = ctypes.c_int
    lib.taser_workspace_size.argtypes = [D, ctypes.POINTER(ctypes.c_size_t)]
    lib.taser_run.restype = ctypes.c_int
    lib.taser_run.argtypes = [D, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    lib.taser_run_static.restype = ctypes.c_int
    lib.taser_run_static.argtypes = [D, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.taser_mixed_workspace_size.restype = ctypes.c_int
    lib.taser_mixed_workspace_size.argtypes = [D, ctypes.POINTER(ctypes.c_size_t)]
    lib.taser_run_mixed.restype = ctypes.c_int
    lib.taser_run_mixed.argtypes = [D, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int32, _P,
                                    ctypes.POINTER(MixedLaunch), _P, ctypes.c_size_t, _P]
    lib.taser_run_prep.restype = ctypes.c_int
    lib.taser_run_prep.argtypes = [D, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    lib.taser_run_solve.restype = ctypes.c_int
    lib.taser_run_solve.argtypes = [D, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    lib.taser_run_tau.restype = ctypes.c_int
    lib.taser_run_tau.argtypes = [D, _P, ctypes.c_size_t, _P, _P]
    lib.taser_fixed_quantize.restype = ctypes.c_int
    lib.taser_fixed_quantize.argtypes = [D, _P, _P, _P, _P, _P, _P]
    lib.taser_fixed_solve.restype = ctypes.c_int
    lib.taser_fixed_solve.argtypes = [D, _P, _P, _P, _P, _P, _P]
    lib.taser_reference_detect.restype = ctypes.c_int
    lib.taser_reference_detect.argtypes = [D, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, _P, _P, _P, _P, _P]
    lib.taser_sdr_detect.restype = ctypes.c_int
    lib.taser_sdr_detect.argtypes = [D, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    lib.taser_jed_channel.restype = ctypes.c_int
    lib.taser_jed_channel.argtypes = [D, _P, _P, _P, _P, _P]
    lib.taser_calibrate.restype = ctypes.c_int
    lib.taser_calibrate.argtypes = [ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double), _P]
    lib.taser_calibrate_elements.restype = ctypes.c_int32
    lib.taser_calibrate_elements.argtypes = []
    U = ctypes.POINTER(UnfoldedDesc)
    lib.taser_unfolded_sizes.restype = ctypes.c_int
    lib.taser_unfolded_sizes.argtypes = [U, ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.POINTER(ctypes.c_size_t)]
    lib.taser_unfolded_forward.restype = ctypes.c_int
    lib.taser_unfolded_forward.argtypes = [U, _P, _P, _P, _P, _P, _P, _P]
    lib.taser_unfolded_backward.restype = ctypes.c_int
    lib.taser_unfolded_backward.argtypes = [U, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]
    _lib = lib
    return lib


def inject_device_error(count: int) -> None:
    """Testing aid: the next ``count`` launching calls fail with
    TASER_ERR_DEVICE before they launch (``taser_debug_inject_device_error``)."""
    _raise(load().taser_debug_inject_device_error(int(count)))


def problem_size(U: int, mod: int) -> int:
    return 2 * U + 1 if mod == QPSK else U + 1


def make_desc(V, B, U, mod, mode=COHERENT, prec=PREC_F32, tau_mode=TAU_SPECTRAL, y_per_H=1,
              t_max=10, flags=0, alpha=0.5) -> Desc:
    return Desc(int(V), int(B), int(U), int(mod), int(mode), int(prec), int(tau_mode),
                int(y_per_H), int(t_max), int(flags), float(alpha))


def check_desc(desc: Desc) -> int:
    return load().taser_check_desc(ctypes.byref(desc))


def _raise(status: int):
    if status != OK:
        raise TaserError(status, load().taser_status_string(status).decode())


def _torch():
    import torch
    return torch


def _need(t, dtype, numel, name):
    torch = _torch()
    if t is None:
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _opt(t, dtype, numel, name):
    return None if t is None else _need(t, dtype, numel, name)


def _stream(device):
    return ctypes.c_void_p(_torch().cuda.current_stream(device).cuda_stream)


def _inputs(desc: Desc, H, y, s0):
    torch = _torch()
    V, B, U = desc.num_vectors, desc.B, desc.U
    if desc.mode == COHERENT:
        ph = _need(H, torch.complex64, (V // max(desc.y_per_H, 1)) * B * U, "H")
        py = _need(y, torch.complex64, V * B, "y")
        ps = None
    else:
        ph = None
        py = _need(y, torch.complex64, V * (U + 1) * B, "Y")
        ps = _need(s0, torch.complex64, V, "s0")
    return ph, py, ps


def build_T(desc: Desc, H, y, s0=None, tau=None):
    """Preprocessing (Section II, Section III-C): returns dict with Tt [V,N,N],
    D [V,N], lam [V], tau [V], status [V].  With desc.tau_mode == TAU_GIVEN
    the given ``tau`` [V] is copied into the result unchanged."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    dev = y.device
    ph, py, ps = _inputs(desc, H, y, s0)
    out = {"Tt": torch.empty((V, N, N), dtype=torch.float32, device=dev),
           "D": torch.empty((V, N), dtype=torch.float32, device=dev),
           "lam": torch.empty((V,), dtype=torch.float32, device=dev),
           "tau": torch.empty((V,), dtype=torch.float32, device=dev),
           "status": torch.empty((V,), dtype=torch.int32, device=dev)}
    if desc.tau_mode == TAU_GIVEN:
        _need(tau, torch.float32, V, "tau")
        out["tau"].copy_(tau)
    st = lib.taser_build_T(ctypes.byref(desc), ph, py, ps,
                           *(ctypes.c_void_p(out[k].data_ptr()) for k in ("Tt", "D", "lam", "tau", "status")),
                           _stream(dev))
    _raise(st)
    return out


def solve(desc: Desc, Tt, D, tau, status):
    """Algorithm 1 main loop: returns packed L~ [V, N(N+1)/2]; ``status`` is
    updated in place."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    P = N * (N + 1) // 2
    L = torch.empty((V, P), dtype=torch.float32, device=Tt.device)
    st = lib.taser_solve(ctypes.byref(desc), _need(Tt, torch.float32, V * N * N, "Tt"),
                         _need(D, torch.float32, V * N, "D"), _need(tau, torch.float32, V, "tau"),
                         ctypes.c_void_p(L.data_ptr()), _need(status, torch.int32, V, "status"),
                         _stream(Tt.device))
    _raise(st)
    return L


def detect(desc: Desc, L, D, want_margin=True):
    """Algorithm 1 output: returns (sbar int8 [V, N-1], margin float32 [V, N-1] or None)."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    sbar = torch.empty((V, N - 1), dtype=torch.int8, device=L.device)
    margin = torch.empty((V, N - 1), dtype=torch.float32, device=L.device) if want_margin else None
    st = lib.taser_detect(ctypes.byref(desc), _need(L, torch.float32, V * N * (N + 1) // 2, "L"),
                          _need(D, torch.float32, V * N, "D"), ctypes.c_void_p(sbar.data_ptr()),
                          None if margin is None else ctypes.c_void_p(margin.data_ptr()),
                          _stream(L.device))
    _raise(st)
    return sbar, margin


def fixed_quantize(desc: Desc, Tt, D, tau):
    """Preprocessing outputs (float32 Tt [V,N,N], D [V,N], tau [V]) to the
    14-bit words of the fixed-point mode: dict That int16 [V,N,N], D int16
    [V,N]."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    out = {"That": torch.empty((V, N, N), dtype=torch.int16, device=Tt.device),
           "D": torch.empty((V, N), dtype=torch.int16, device=Tt.device)}
    _raise(lib.taser_fixed_quantize(ctypes.byref(desc), _need(Tt, torch.float32, V * N * N, "Tt"),
                                    _need(D, torch.float32, V * N, "D"), _need(tau, torch.float32, V, "tau"),
                                    _need(out["That"], torch.int16, V * N * N, "That"),
                                    _need(out["D"], torch.int16, V * N, "Dq"), _stream(Tt.device)))
    return out


def fixed_solve(desc: Desc, That, Dq, status):
    """Fixed-point Algorithm 1 on words: dict L int16 [V, N(N+1)/2] (packed
    words), sbar int8 [V, N-1], status (``status`` is updated in place)."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    out = {"L": torch.empty((V, N * (N + 1) // 2), dtype=torch.int16, device=That.device),
           "sbar": torch.empty((V, N - 1), dtype=torch.int8, device=That.device), "status": status}
    _raise(lib.taser_fixed_solve(ctypes.byref(desc), _need(That, torch.int16, V * N * N, "That"),
                                 _need(Dq, torch.int16, V * N, "Dq"),
                                 _need(out["L"], torch.int16, V * N * (N + 1) // 2, "L"),
                                 _need(out["sbar"], torch.int8, V * (N - 1), "sbar"),
                                 _need(status, torch.int32, V, "status"), _stream(That.device)))
    return out


REF_MF, REF_MMSE, REF_ML, REF_KBEST = 0, 1, 2, 3


def reference_detect(desc: Desc, kind: int, H, y, K: int = 5, n0: float = 0.0, want_soft=False):
    """Reference detectors (``taser_reference_detect``): returns (sbar int8
    [V, N-1], soft or None); soft is the estimate [V, N-1] (MF, MMSE) or the
    residual [V] (ML, K-best)."""
    torch = _torch()
    lib = load()
    V, M = desc.num_vectors, problem_size(desc.U, desc.mod) - 1
    dev = y.device
    ph, py, _ = _inputs(desc, H, y, None)
    sbar = torch.empty((V, M), dtype=torch.int8, device=dev)
    soft = None
    if want_soft:
        soft = torch.empty((V, M) if kind in (REF_MF, REF_MMSE) else (V,), dtype=torch.float32, device=dev)
    _raise(lib.taser_reference_detect(ctypes.byref(desc), int(kind), int(K), float(n0), ph, py,
                                      _need(sbar, torch.int8, V * M, "sbar"),
                                      None if soft is None else ctypes.c_void_p(soft.data_ptr()), _stream(dev)))
    return sbar, soft


def sdr_detect(desc: Desc, Tt, D=None, status=None, want_X=False):
    """Exact SDR detector of eq. (7) (``taser_sdr_detect``) on T = D T~ D
    (``Tt``, ``D`` as ``build_T`` returns them) or, with ``D=None``, on
    ``Tt`` = T itself (float32).  Returns dict sbar [V, N-1], objective [V],
    gap [V], iterations [V] and, with ``want_X``, X [V, N, N] (float64)."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    dev = Tt.device
    out = {"sbar": torch.empty((V, N - 1), dtype=torch.int8, device=dev),
           "objective": torch.empty((V,), dtype=torch.float64, device=dev),
           "gap": torch.empty((V,), dtype=torch.float64, device=dev),
           "iterations": torch.empty((V,), dtype=torch.int32, device=dev)}
    if want_X:
        out["X"] = torch.empty((V, N, N), dtype=torch.float64, device=dev)
    _raise(lib.taser_sdr_detect(ctypes.byref(desc), _need(Tt, torch.float32, V * N * N, "Tt"),
                                _opt(D, torch.float32, V * N, "D"), _opt(status, torch.int32, V, "status"),
                                ctypes.c_void_p(out["sbar"].data_ptr()), ctypes.c_void_p(out["objective"].data_ptr()),
                                ctypes.c_void_p(out["gap"].data_ptr()),
                                ctypes.c_void_p(out["X"].data_ptr()) if want_X else None,
                                ctypes.c_void_p(out["iterations"].data_ptr()), _stream(dev)))
    return out


def jed_channel(desc: Desc, Y, s0, sbar):
    """Channel estimate h = Y [s0; s_r] of joint detection (eq. (4)) from the
    detected symbols ``sbar`` [V, N-1]; returns complex64 [V, B]."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    h = torch.empty((V, desc.B), dtype=torch.complex64, device=Y.device)
    st = lib.taser_jed_channel(ctypes.byref(desc), _need(Y, torch.complex64, V * (desc.U + 1) * desc.B, "Y"),
                               _need(s0, torch.complex64, V, "s0"), _need(sbar, torch.int8, V * (N - 1), "sbar"),
                               ctypes.c_void_p(h.data_ptr()), _stream(Y.device))
    _raise(st)
    return h


def workspace_size(desc: Desc) -> int:
    """Bytes of device workspace ``run`` needs for ``desc``."""
    n = ctypes.c_size_t(0)
    _raise(load().taser_workspace_size(ctypes.byref(desc), ctypes.byref(n)))
    return int(n.value)


_ws_cache = {}


def _workspace(nbytes, device):
    """A cached device buffer of at least ``nbytes`` per device (torch-allocated)."""
    torch = _torch()
    key = (device.type, device.index if device.index is not None else torch.cuda.current_device())
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def run(desc: Desc, H, y, s0=None, tau=None, want_margin=False, want_L=False, out=None, ws=None):
    """The fused detector.  Returns dict sbar, status (+ margin, L when
    requested).  ``out`` may hold preallocated tensors to reuse; ``ws`` a
    uint8 device workspace (a cached one is used otherwise)."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    dev = y.device
    ph, py, ps = _inputs(desc, H, y, s0)
    pt = _need(tau, torch.float32, V, "tau") if desc.tau_mode == TAU_GIVEN else None
    res = out if out is not None else {}
    if "sbar" not in res:
        res["sbar"] = torch.empty((V, N - 1), dtype=torch.int8, device=dev)
        res["status"] = torch.empty((V,), dtype=torch.int32, device=dev)
    if want_margin and "margin" not in res:
        res["margin"] = torch.empty((V, N - 1), dtype=torch.float32, device=dev)
    if want_L and "L" not in res:
        res["L"] = torch.empty((V, N * (N + 1) // 2), dtype=torch.float32, device=dev)
    nbytes = workspace_size(desc)
    if ws is None:
        ws = _workspace(nbytes, dev)
    if ws.dtype != torch.uint8 or not ws.is_cuda or ws.numel() < nbytes:
        raise ValueError(f"workspace must be a uint8 CUDA tensor of at least {nbytes} bytes")
    st = lib.taser_run(ctypes.byref(desc), ph, py, ps, pt,
                       _need(res["sbar"], torch.int8, V * (N - 1), "sbar"),
                       _opt(res.get("margin") if want_margin else None, torch.float32, V * (N - 1), "margin"),
                       _need(res["status"], torch.int32, V, "status"),
                       _opt(res.get("L") if want_L else None, torch.float32, V * N * (N + 1) // 2, "L"),
                       ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                       _stream(dev))
    _raise(st)
    return res


def _outputs(desc, dev, res, want_margin, want_L):
    torch = _torch()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    if "sbar" not in res:
        res["sbar"] = torch.empty((V, N - 1), dtype=torch.int8, device=dev)
    if "status" not in res:
        res["status"] = torch.empty((V,), dtype=torch.int32, device=dev)
    if want_margin and "margin" not in res:
        res["margin"] = torch.empty((V, N - 1), dtype=torch.float32, device=dev)
    if want_L and "L" not in res:
        res["L"] = torch.empty((V, N * (N + 1) // 2), dtype=torch.float32, device=dev)
    return res


def _ws_for(desc, dev, ws):
    torch = _torch()
    nbytes = workspace_size(desc)
    if ws is None:
        ws = _workspace(nbytes, dev)
    if ws.dtype != torch.uint8 or not ws.is_cuda or ws.numel() < nbytes:
        raise ValueError(f"workspace must be a uint8 CUDA tensor of at least {nbytes} bytes")
    return ws


def run_prep(desc: Desc, H, y, s0=None, tau=None, out=None, ws=None):
    """First stage of ``run``: T, preconditioning and step size into the
    workspace; returns the ``out`` dict (status filled in)."""
    torch = _torch()
    lib = load()
    V = desc.num_vectors
    dev = y.device
    ph, py, ps = _inputs(desc, H, y, s0)
    pt = _need(tau, torch.float32, V, "tau") if desc.tau_mode == TAU_GIVEN else None
    res = _outputs(desc, dev, out if out is not None else {}, False, False)
    ws = _ws_for(desc, dev, ws)
    st = lib.taser_run_prep(ctypes.byref(desc), ph, py, ps, pt,
                            _need(res["status"], torch.int32, V, "status"),
                            ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), _stream(dev))
    _raise(st)
    return res


def run_solve(desc: Desc, out, want_margin=False, want_L=False, ws=None, device=None):
    """Second stage of ``run``: Algorithm 1 and slicing from the workspace the
    matching ``run_prep`` filled."""
    torch = _torch()
    lib = load()
    V, N = desc.num_vectors, problem_size(desc.U, desc.mod)
    dev = device if device is not None else out["status"].device
    res = _outputs(desc, dev, out, want_margin, want_L)
    ws = _ws_for(desc, dev, ws)
    st = lib.taser_run_solve(ctypes.byref(desc), _need(res["sbar"], torch.int8, V * (N - 1), "sbar"),
                             _opt(res.get("margin") if want_margin else None, torch.float32, V * (N - 1), "margin"),
                             _need(res["status"], torch.int32, V, "status"),
                             _opt(res.get("L") if want_L else None, torch.float32, V * N * (N + 1) // 2, "L"),
                             ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), _stream(dev))
    _raise(st)
    return res


def run_tau(desc: Desc, ws, device=None):
    """Step sizes tau [V] (float32) of a workspace ``run_prep`` filled."""
    torch = _torch()
    lib = load()
    dev = device if device is not None else ws.device
    tau = torch.empty(desc.num_vectors, dtype=torch.float32, device=dev)
    st = lib.taser_run_tau(ctypes.byref(desc), ctypes.c_void_p(ws.data_ptr()),
                           ctypes.c_size_t(ws.numel()), ctypes.c_void_p(tau.data_ptr()), _stream(dev))
    _raise(st)
    return tau


def calibrate(kind: int, iters: int, out=None, device=None):
    """Launch calibration kernel ``kind`` (0 float32 FMA, 1 BF16 MFMA, 2 float32
    MFMA); returns (out tensor, flops of the launch).  The caller times it."""
    torch = _torch()
    lib = load()
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty(int(lib.taser_calibrate_elements()), dtype=torch.float32, device=dev)
    fl = ctypes.c_double(0.0)
    _raise(lib.taser_calibrate(int(kind), int(iters), ctypes.c_void_p(out.data_ptr()), ctypes.byref(fl),
                               _stream(dev)))
    return out, fl.value


MIXED_STRIDE = 64


def run_mixed(desc: Desc, Bv, Uv, modv, H_off, y_off, H, y, tau=None, want_margin=False,
              blocks=None, out=None, ws=None, waves=None, single=False, concurrent=False):
    """Mixed-size coherent batch in one call (``taser_run_mixed``).
    Bv, Uv, modv: int32 [V]; H_off, y_off: int64 [V] (complex elements);
    H, y: flat complex64 device tensors.  Launch choices (e.g. from the
    autotuner): ``blocks`` grid per bucket (3 ints, 0 = default), ``waves``
    register budget per bucket (3 ints, 0 default, 1 alternative),
    ``single`` every bucket in one launch, ``concurrent`` the bucket kernels
    on three streams.  Returns dict with sbar int8
    [V, 64] (first N_v - 1 entries valid), status (+ margin)."""
    torch = _torch()
    lib = load()
    V = desc.num_vectors
    dev = y.device
    for name, t, dt in (("B", Bv, torch.int32), ("U", Uv, torch.int32), ("mod", modv, torch.int32),
                        ("H_off", H_off, torch.int64), ("y_off", y_off, torch.int64)):
        _need(t, dt, V, name)
    for name, t in (("H", H), ("y", y)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex64 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous complex64 CUDA tensor")
    pt = _need(tau, torch.float32, V, "tau") if desc.tau_mode == TAU_GIVEN else None
    res = out if out is not None else {}
    if "sbar" not in res:
        res["sbar"] = torch.empty((V, MIXED_STRIDE), dtype=torch.int8, device=dev)
        res["status"] = torch.empty((V,), dtype=torch.int32, device=dev)
    if want_margin and "margin" not in res:
        res["margin"] = torch.empty((V, MIXED_STRIDE), dtype=torch.float32, device=dev)
    n = ctypes.c_size_t(0)
    _raise(lib.taser_mixed_workspace_size(ctypes.byref(desc), ctypes.byref(n)))
    if ws is None:
        ws = _workspace(int(n.value), dev)
    if ws.dtype != torch.uint8 or ws.numel() < n.value:
        raise ValueError(f"workspace must be a uint8 CUDA tensor of at least {n.value} bytes")
    launch = MixedLaunch()
    if blocks is not None:
        for i, b in enumerate(blocks):
            launch.blocks[i] = int(b)
    if waves is not None:
        for i, w in enumerate(waves):
            launch.waves[i] = int(w)
    launch.single_launch = 1 if single else 0
    launch.concurrent = 1 if concurrent else 0
    st = lib.taser_run_mixed(ctypes.byref(desc), *(ctypes.c_void_p(t.data_ptr()) for t in (Bv, Uv, modv, H_off, y_off, H, y)),
                             pt, ctypes.c_void_p(res["sbar"].data_ptr()),
                             ctypes.c_void_p(res["margin"].data_ptr()) if want_margin else None,
                             ctypes.c_int32(MIXED_STRIDE), ctypes.c_void_p(res["status"].data_ptr()),
                             ctypes.byref(launch), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                             _stream(dev))
    _raise(st)
    return res


# ---- Unfolded TASER (per-iteration step sizes) ----------------------------

def _unf_desc(Tt, alpha, ckpt_every, literal_last):
    torch = _torch()
    if Tt.dim() != 3 or Tt.shape[1] != Tt.shape[2]:
        raise ValueError("Tt must be [V, N, N]")
    if Tt.dtype not in (torch.float32, torch.float64):
        raise ValueError("Tt must be float32 or float64")
    V, N = Tt.shape[0], Tt.shape[1]
    t_max = alpha.numel()
    real = REAL_F64 if Tt.dtype == torch.float64 else REAL_F32
    flags = FLAG_LITERAL_LAST if literal_last else 0
    if ckpt_every:
        return UnfoldedDesc(V, N, t_max, real, int(ckpt_every), flags)
    # default: a checkpoint every 2 iterations.  The backward keeps c + 1
    # states in LDS; on gfx950 c = 2 gave the fastest backward (1.5x faster
    # than c = 4 ~ sqrt(20), whose LDS footprint halves the waves per CU;
    # c = 1 waits on a checkpoint load from HBM every step), and the
    # checkpoints cost V * t_max/2 * N(N+1)/2 values of HBM.
    c = min(2, t_max)
    return UnfoldedDesc(V, N, t_max, real, c, flags)


def unfolded_sizes(u: UnfoldedDesc):
    """(checkpoint elements, backward workspace bytes) for ``u``."""
    ck, ws = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _raise(load().taser_unfolded_sizes(ctypes.byref(u), ctypes.byref(ck), ctypes.byref(ws)))
    return int(ck.value), int(ws.value)


def unfolded_forward(Tt, D, lam, alpha, ckpt_every=None, literal_last=False):
    """Algorithm 1 with tau_t = alpha[t] / lam.  Tt [V,N,N], D [V,N], lam [V],
    alpha [t_max], all float32 or all float64 on one device.  Returns
    (L packed [V, N(N+1)/2], checkpoints, desc) for ``unfolded_backward``."""
    torch = _torch()
    lib = load()
    u = _unf_desc(Tt, alpha, ckpt_every, literal_last)
    V, N, dt = u.num_vectors, u.N, Tt.dtype
    n_ck, _ = unfolded_sizes(u)
    ckpt = torch.empty((max(n_ck, 1),), dtype=dt, device=Tt.device)
    L = torch.empty((V, N * (N + 1) // 2), dtype=dt, device=Tt.device)
    st = lib.taser_unfolded_forward(ctypes.byref(u), _need(Tt, dt, V * N * N, "Tt"),
                                    _need(D, dt, V * N, "D"), _need(lam, dt, V, "lam"),
                                    _need(alpha, dt, u.t_max, "alpha"),
                                    ctypes.c_void_p(ckpt.data_ptr()), ctypes.c_void_p(L.data_ptr()),
                                    _stream(Tt.device))
    _raise(st)
    return L, ckpt, u


def unfolded_backward(u: UnfoldedDesc, Tt, D, lam, alpha, ckpt, dL):
    """dLoss/dalpha [t_max] (summed over the batch) given dL = dLoss/dL_out."""
    torch = _torch()
    lib = load()
    V, N, dt = u.num_vectors, u.N, Tt.dtype
    _, ws_bytes = unfolded_sizes(u)
    ws = torch.empty((max(ws_bytes, 8),), dtype=torch.uint8, device=Tt.device)
    dalpha = torch.empty((u.t_max,), dtype=dt, device=Tt.device)
    st = lib.taser_unfolded_backward(ctypes.byref(u), _need(Tt, dt, V * N * N, "Tt"),
                                     _need(D, dt, V * N, "D"), _need(lam, dt, V, "lam"),
                                     _need(alpha, dt, u.t_max, "alpha"),
                                     ctypes.c_void_p(ckpt.data_ptr()),
                                     _need(dL, dt, V * N * (N + 1) // 2, "dL"),
                                     ctypes.c_void_p(dalpha.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(Tt.device))
    _raise(st)
    return dalpha
