"""Launch-configuration autotuner for the mixed-size batch path.

The tunable knob is the grid of each size bucket (N-1 <= 16, <= 32, <= 64):
0 = one one-wave workgroup per vector of the batch (the library default),
n > 0 = a persistent grid of n workgroups walking the bucket's vector list.
The persistent kernel saves workgroup launches but carries its loop's state
in registers; which wins depends on the bucket and the batch.
``tune_mixed`` times candidate grids on the device for one bucket at
a time (coordinate descent, the other buckets at their current best), keeps
the fastest, and caches the result in a JSON file keyed by GPU architecture,
bucket, precision and t_max.  Timing uses HIP events on the launch stream.
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


def cache_key(bucket, prec, t_max, num_vectors):
    """Key of a tuned grid: architecture, bucket, precision, t_max and the
    batch size class (log2 of the vector count: the best persistent grid
    depends on how many vectors each bucket holds)."""
    size_class = max(int(num_vectors), 1).bit_length()
    return f"{_arch()}|mixed|b{bucket}|p{prec}|t{t_max}|v2^{size_class}"


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


def cached_blocks(prec, t_max, num_vectors, path=DEFAULT_CACHE):
    """Tuned grid per bucket from the cache (0 = library default)."""
    cache = load_cache(path)
    return [int(cache.get(cache_key(b, prec, t_max, num_vectors), {}).get("blocks", 0))
            for b in range(3)]


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


def tune_mixed(desc, args, candidates=CANDIDATES, path=DEFAULT_CACHE, reps=3, sweeps=1, rounds=15):
    """Tune the per-bucket grid of ``run_mixed(desc, *args)`` and store it.

    Coordinate descent over the buckets with short timings proposes a
    winner (a candidate equal to the current best is not timed again).  The
    winner and the default are then timed interleaved over ``rounds``
    rounds; the winner is adopted only if its median beats the default's
    p10 (faster than the default's spread), otherwise the default is kept.
    Returns (blocks, {"default": stats, "tuned": stats, "adopted": bool,
    "proposed": blocks}, trace)."""
    import paper_1609_01797_amd as taser
    out = {}

    def call(blocks):
        return lambda: taser.run_mixed(desc, *args, blocks=blocks, out=out)

    best = [0, 0, 0]
    best_ms = _time_call(call(best), reps)
    trace = [{"blocks": list(best), "ms": best_ms}]
    for _ in range(sweeps):
        for b in range(3):
            for c in candidates:
                if c == best[b]:
                    continue
                trial = list(best)
                trial[b] = c
                ms = _time_call(call(trial), reps)
                trace.append({"blocks": trial, "ms": ms})
                if ms < best_ms:
                    best_ms, best = ms, trial
    default = [0, 0, 0]
    if best == default:
        st, _ = compare(call(default), call(default), rounds=max(rounds // 3, 3), reps=reps)
        report = {"default": st, "tuned": st, "adopted": False, "proposed": default}
    else:
        st_d, st_t = compare(call(default), call(best), rounds=rounds, reps=reps)
        adopted = st_t["median_ms"] < st_d["p10_ms"]
        report = {"default": st_d, "tuned": st_t, "adopted": adopted, "proposed": list(best)}
        if not adopted:
            best = default
    cache = load_cache(path)
    for b in range(3):
        cache[cache_key(b, desc.prec, desc.t_max, desc.num_vectors)] = {
            "blocks": best[b], "median_ms": report["tuned" if report["adopted"] else "default"]["median_ms"]}
    save_cache(cache, path)
    return best, report, trace
