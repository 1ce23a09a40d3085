"""Seeded synthetic inputs for TASER: channels, symbols and noise.

This module is shared by the FP64 oracle's tests, the GPU tests and the
benchmark.  It holds no detector arithmetic: it only draws random channels,
transmit symbols and noise in the distributions the paper simulates
(i.i.d. flat Rayleigh fading, Section V-A) and returns them as complex64
arrays.  Every consumer (the oracle, the HIP path) reads the very same
complex64 values.

Conventions (the paper fixes none of them numerically):

* QPSK symbols are {+-1 +- 1j} and BPSK symbols are {+-1}: the real-valued
  reformulation of eq. (2) needs the real and imaginary parts of every
  symbol in {-1, +1}, so no 1/sqrt(2) normalisation is applied.
  Es = 2 (QPSK) or 1 (BPSK).
* SNR is per receive antenna.  Coherent MU-MIMO (Section II-A):
  SNR = E||Hs||^2 / E||n||^2 = U*Es/N0.  SIMO block fading (Section II-B):
  SNR = Es/N0.  So N0 = U*Es*10^(-SNR/10) and N0 = Es*10^(-SNR/10).
* Joint channel estimation and detection follows the paper's model
  Y = h s^H + N (Section II-B) literally: the returned ``s`` holds the
  paper's s_0..s_K, with s_0 the known pilot (1 for BPSK, 1+1j for QPSK).
  Y is stored slot-major: Y[v, k, b] is antenna b in time slot k.

Seeds: ``seed_for(config, snr_index, shard)`` gives the base recipe
160901797 + 10000*config + 100*snr_index + shard for numpy's PCG64.
"""
from __future__ import annotations

import numpy as np

BPSK = 1
QPSK = 2

SEED_BASE = 160901797


def seed_for(config: int, snr_index: int = 0, shard: int = 0) -> int:
    """Seed recipe for workload ``config`` (1-based), SNR point and shard."""
    return SEED_BASE + 10000 * int(config) + 100 * int(snr_index) + int(shard)


def symbol_energy(mod: int) -> float:
    if mod == QPSK:
        return 2.0
    if mod == BPSK:
        return 1.0
    raise ValueError(f"unknown modulation {mod}")


def noise_variance(snr_db: float, mod: int, users: int = 1) -> float:
    """N0 for a per-receive-antenna SNR (see module docstring)."""
    return float(users * symbol_energy(mod) * 10.0 ** (-float(snr_db) / 10.0))


def _cn(rng: np.random.Generator, shape, var: float) -> np.ndarray:
    """Circularly-symmetric complex Gaussian with E|x|^2 = var (drawn in FP64)."""
    sd = np.sqrt(var / 2.0)
    return sd * rng.standard_normal(shape) + 1j * (sd * rng.standard_normal(shape))


def _symbols(rng: np.random.Generator, shape, mod: int) -> np.ndarray:
    re = rng.integers(0, 2, size=shape) * 2 - 1
    if mod == BPSK:
        return re.astype(np.complex128)
    im = rng.integers(0, 2, size=shape) * 2 - 1
    return re + 1j * im


def pilot_symbol(mod: int) -> complex:
    return complex(1.0, 1.0) if mod == QPSK else complex(1.0, 0.0)


def gen_mimo(B: int, U: int, mod: int, num_H: int, y_per_H: int, snr_db: float,
             seed: int, noiseless: bool = False) -> dict:
    """Coherent MU-MIMO uplink y = H s + n (Section II-A).

    Returns a dict with
      H : complex64 [num_H, B, U]   (vector v uses H[v // y_per_H])
      s : complex64 [V, U]          transmitted symbols, V = num_H * y_per_H
      y : complex64 [V, B]
      N0: float
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    V = num_H * y_per_H
    H = _cn(rng, (num_H, B, U), 1.0)
    s = _symbols(rng, (V, U), mod)
    N0 = noise_variance(snr_db, mod, U)
    n = _cn(rng, (V, B), N0)
    Hv = np.repeat(H, y_per_H, axis=0)
    y = np.einsum("vbu,vu->vb", Hv, s)
    if not noiseless:
        y = y + n
    return {"H": H.astype(np.complex64), "s": s.astype(np.complex64),
            "y": y.astype(np.complex64), "N0": N0, "B": B, "U": U, "mod": mod,
            "y_per_H": y_per_H}


def gen_jed(B: int, K: int, mod: int, num_blocks: int, snr_db: float, seed: int,
            noiseless: bool = False) -> dict:
    """SIMO block fading Y = h s^H + N over K+1 slots (Section II-B).

    Returns a dict with
      Y : complex64 [V, K+1, B]  slot-major received block
      s : complex64 [V, K+1]     the paper's s (s[:, 0] is the pilot s_0)
      s0: complex64 [V]          pilot symbols
      h : complex64 [V, B]
      N0: float
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    V = num_blocks
    h = _cn(rng, (V, B), 1.0)
    s = _symbols(rng, (V, K + 1), mod)
    s[:, 0] = pilot_symbol(mod)
    N0 = noise_variance(snr_db, mod, 1)
    n = _cn(rng, (V, K + 1, B), N0)
    # Y[:, b, k] = h_b * conj(s_k)  ->  slot-major Y[v, k, b]
    Y = np.conj(s)[:, :, None] * h[:, None, :]
    if not noiseless:
        Y = Y + n
    return {"Y": Y.astype(np.complex64), "s": s.astype(np.complex64),
            "s0": s[:, 0].astype(np.complex64), "h": h.astype(np.complex64),
            "N0": N0, "B": B, "K": K, "mod": mod}


MIXED_CLASSES = ((64, 8, BPSK), (64, 8, QPSK), (128, 16, BPSK), (128, 16, QPSK),
                 (256, 32, BPSK), (256, 32, QPSK))


def gen_mixed(num_vectors: int, snr_db: float, seed: int,
              classes=MIXED_CLASSES) -> dict:
    """Mixed-size batch: each vector draws (B, U, mod) uniformly from ``classes``
    and its own Rayleigh channel.  Vectors are returned unsorted, packed back to
    back: H_flat holds every vector's B*U entries and y_flat its B entries.

    Returns a dict with
      cls    : int32 [V]         index into ``classes``
      B, U, mod : int32 [V]
      H_off, y_off : int64 [V]   element offsets into H_flat / y_flat
      H_flat : complex64 [sum B*U]
      y_flat : complex64 [sum B]
      s      : list of complex64 [U_v] arrays
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cls = rng.integers(0, len(classes), size=num_vectors).astype(np.int32)
    Bs = np.array([classes[c][0] for c in cls], dtype=np.int32)
    Us = np.array([classes[c][1] for c in cls], dtype=np.int32)
    mods = np.array([classes[c][2] for c in cls], dtype=np.int32)
    H_off = np.zeros(num_vectors, dtype=np.int64)
    y_off = np.zeros(num_vectors, dtype=np.int64)
    H_off[1:] = np.cumsum(Bs.astype(np.int64) * Us)[:-1]
    y_off[1:] = np.cumsum(Bs.astype(np.int64))[:-1]
    H_flat = np.empty(int((Bs.astype(np.int64) * Us).sum()), dtype=np.complex64)
    y_flat = np.empty(int(Bs.sum()), dtype=np.complex64)
    s_list = []
    for v in range(num_vectors):
        B, U, mod = int(Bs[v]), int(Us[v]), int(mods[v])
        H = _cn(rng, (B, U), 1.0)
        s = _symbols(rng, (U,), mod)
        n = _cn(rng, (B,), noise_variance(snr_db, mod, U))
        H_flat[H_off[v]:H_off[v] + B * U] = H.astype(np.complex64).ravel()
        y_flat[y_off[v]:y_off[v] + B] = (H @ s + n).astype(np.complex64)
        s_list.append(s.astype(np.complex64))
    return {"cls": cls, "B": Bs, "U": Us, "mod": mods, "H_off": H_off, "y_off": y_off,
            "H_flat": H_flat, "y_flat": y_flat, "s": s_list}


def gen_training_batch(B: int, U: int, mod: int, batch: int, snr_lo: float,
                       snr_hi: float, seed: int) -> dict:
    """Training batch for the unfolded detector: every sample draws its own
    channel and its own SNR uniformly in [snr_lo, snr_hi] dB (counter-based:
    batch i of a run uses seed base+i, so a resumed run replays the batches)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = _cn(rng, (batch, B, U), 1.0)
    s = _symbols(rng, (batch, U), mod)
    snr = rng.uniform(snr_lo, snr_hi, size=batch)
    N0 = U * symbol_energy(mod) * 10.0 ** (-snr / 10.0)
    n = _cn(rng, (batch, B), 1.0) * np.sqrt(N0)[:, None]
    y = np.einsum("vbu,vu->vb", H, s) + n
    return {"H": H.astype(np.complex64), "s": s.astype(np.complex64),
            "y": y.astype(np.complex64), "snr_db": snr}


def gen_training_batch_torch(B: int, U: int, mod: int, batch: int, snr_lo: float,
                             snr_hi: float, seed: int, device) -> dict:
    """``gen_training_batch`` drawn on ``device`` with torch's generator (same
    distributions, not the same numbers): fresh training data for long
    training runs without host-side generation.  Returns complex64 tensors
    H [batch, B, U], s [batch, U], y [batch, B] and snr_db [batch]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))

    def cn(shape, var):
        sd = torch.sqrt(torch.as_tensor(var, dtype=torch.float32, device=device) / 2.0)
        re = torch.randn(shape, generator=g, device=device)
        im = torch.randn(shape, generator=g, device=device)
        if sd.dim():
            sd = sd.reshape(sd.shape + (1,) * (len(shape) - sd.dim()))
        return torch.complex(re * sd, im * sd)

    def bits(shape):
        return (torch.randint(0, 2, shape, generator=g, device=device) * 2 - 1).float()

    H = cn((batch, B, U), 1.0)
    re = bits((batch, U))
    im = bits((batch, U)) if mod == QPSK else torch.zeros_like(re)
    s = torch.complex(re, im)
    snr = snr_lo + (snr_hi - snr_lo) * torch.rand(batch, generator=g, device=device)
    N0 = U * symbol_energy(mod) * 10.0 ** (-snr / 10.0)
    y = (H * s[:, None, :]).sum(-1) + cn((batch, B), N0)
    return {"H": H, "s": s, "y": y, "snr_db": snr}
