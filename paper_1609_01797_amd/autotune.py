"""Launch-configuration autotuner for the mixed-size batch path.

The choices, per size bucket (N-1 <= 16, <= 32, <= 64), are the grid
(0 = one one-wave workgroup per vector of the batch, the library default;
n > 0 = a persistent grid of n workgroups walking the bucket's vector list)
and the register budget of the one-workgroup-per-vector kernel (0 = the
default build, 1 = the alternative: more waves per SIMD for one and four
column tiles, fewer for two); and, for the whole batch, a single launch of
one kernel over one work queue with the registers of the largest size, or
the bucket kernels on three streams at once (``concurrent``).
``tune_mixed`` searches them on the device by coordinate descent (one
choice at a time, the others at their current best, short timings), then
times the proposal and the default interleaved and adopts the proposal only
if its median beats the default's p10.  The result is cached in a JSON file
keyed by GPU architecture, precision, t_max and batch-size class.  Timing
uses HIP events on the launch stream.
"""
from __future__ import annotations

import json
import os
import threading

_LOCK = threading.Lock()
CANDIDATES = (0, 1024, 2048, 4096, 8192, 16384)
DEFAULT_CACHE = os.environ.get("TASER_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "taser_autotune.json"))


def _arch():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def cache_key(prec, t_max, num_vectors):
    """Key of a tuned configuration: architecture, precision, t_max and the
    batch size class (log2 of the vector count: the best grids depend on how
    many vectors each bucket holds)."""
    size_class = max(int(num_vectors), 1).bit_length()
    return f"{_arch()}|mixed|p{prec}|t{t_max}|v2^{size_class}"


def load_cache(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=DEFAULT_CACHE):
    with _LOCK:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


DEFAULT = {"blocks": [0, 0, 0], "waves": [0, 0, 0], "single": 0, "concurrent": 0}


def cached_config(prec, t_max, num_vectors, path=DEFAULT_CACHE):
    """Tuned launch choices from the cache (the defaults when absent)."""
    rec = load_cache(path).get(cache_key(prec, t_max, num_vectors))
    if not rec:
        return dict(DEFAULT)
    return {"blocks": list(rec["blocks"]), "waves": list(rec["waves"]), "single": int(rec["single"]),
            "concurrent": int(rec.get("concurrent", 0))}


def _time_call(fn, reps=5):
    """Mean milliseconds of ``reps`` back-to-back calls (after one warm-up)."""
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _stats(ms):
    import numpy as np
    ms = np.asarray(ms, dtype=float)
    return {"median_ms": float(np.median(ms)), "p10_ms": float(np.percentile(ms, 10)),
            "p90_ms": float(np.percentile(ms, 90)), "samples": int(ms.size)}


def compare(fn_a, fn_b, rounds=15, reps=3):
    """Time two configurations interleaved (a, b, a, b, ...) so that drift of
    the device clock or of other load affects both alike; returns the
    statistics of each (median, p10, p90 of ``rounds`` timings)."""
    ta, tb = [], []
    for _ in range(rounds):
        ta.append(_time_call(fn_a, reps))
        tb.append(_time_call(fn_b, reps))
    return _stats(ta), _stats(tb)


def _key(cfg):
    return (tuple(cfg["blocks"]), tuple(cfg["waves"]), cfg["single"], cfg.get("concurrent", 0))


def tune_mixed(desc, args, candidates=CANDIDATES, path=DEFAULT_CACHE, reps=3, sweeps=1, rounds=15):
    """Tune the launch choices of ``run_mixed(desc, *args)`` and store them.

    Coordinate descent with short timings proposes a configuration (a choice
    equal to the current best is not timed again); the proposal and the
    default are then timed interleaved over ``rounds`` rounds and the
    proposal is adopted only if its median beats the default's p10.
    Returns (config, {"default": stats, "tuned": stats, "adopted": bool,
    "proposed": config}, trace)."""
    import paper_1609_01797_amd as taser
    out = {}

    def call(cfg):
        return lambda: taser.run_mixed(desc, *args, blocks=cfg["blocks"], waves=cfg["waves"],
                                       single=bool(cfg["single"]),
                                       concurrent=bool(cfg.get("concurrent", 0)), out=out)

    def variant(cfg, field, b, value):
        new = {"blocks": list(cfg["blocks"]), "waves": list(cfg["waves"]), "single": cfg["single"],
               "concurrent": cfg.get("concurrent", 0)}
        if field in ("single", "concurrent"):
            new[field] = value
        else:
            new[field][b] = value
        return new

    best = dict(DEFAULT, blocks=[0, 0, 0], waves=[0, 0, 0])
    best_ms = _time_call(call(best), reps)
    seen = {_key(best): best_ms}
    trace = [{"config": best, "ms": best_ms}]
    choices = [("single", 0, (0, 1)), ("concurrent", 0, (0, 1))]
    for b in range(3):
        choices += [("blocks", b, candidates), ("waves", b, (0, 1))]
    for _ in range(sweeps):
        for field, b, values in choices:
            for value in values:
                trial = variant(best, field, b, value)
                if _key(trial) in seen:
                    continue
                ms = _time_call(call(trial), reps)
                seen[_key(trial)] = ms
                trace.append({"config": trial, "ms": ms})
                if ms < best_ms:
                    best_ms, best = ms, trial
    default = dict(DEFAULT, blocks=[0, 0, 0], waves=[0, 0, 0])
    if _key(best) == _key(default):
        st, _ = compare(call(default), call(default), rounds=max(rounds // 3, 3), reps=reps)
        report = {"default": st, "tuned": st, "adopted": False, "proposed": default}
    else:
        st_d, st_t = compare(call(default), call(best), rounds=rounds, reps=reps)
        adopted = st_t["median_ms"] < st_d["p10_ms"]
        report = {"default": st_d, "tuned": st_t, "adopted": adopted, "proposed": best}
        if not adopted:
            best = default
    cache = load_cache(path)
    cache[cache_key(desc.prec, desc.t_max, desc.num_vectors)] = dict(
        best, median_ms=report["tuned" if report["adopted"] else "default"]["median_ms"])
    save_cache(cache, path)
    return best, report, trace
