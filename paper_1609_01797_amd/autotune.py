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


def cache_key(bucket, prec, t_max):
    return f"{_arch()}|mixed|b{bucket}|p{prec}|t{t_max}"


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


def cached_blocks(prec, t_max, path=DEFAULT_CACHE):
    """Tuned grid per bucket from the cache (0 = library default)."""
    cache = load_cache(path)
    return [int(cache.get(cache_key(b, prec, t_max), {}).get("blocks", 0)) for b in range(3)]


def _time_call(fn, reps=5):
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


def tune_mixed(desc, args, candidates=CANDIDATES, path=DEFAULT_CACHE, reps=5, sweeps=1):
    """Tune the per-bucket persistent grid of ``run_mixed(desc, *args)`` and
    store it.  Returns (best blocks, best ms, default ms, trace)."""
    import paper_1609_01797_amd as taser
    out = {}
    ws = None
    best = [0, 0, 0]

    def call(blocks):
        return lambda: taser.run_mixed(desc, *args, blocks=blocks, out=out, ws=ws)

    default_ms = _time_call(call([0, 0, 0]), reps)
    best_ms = default_ms
    trace = [{"blocks": [0, 0, 0], "ms": default_ms}]
    for _ in range(sweeps):
        for b in range(3):
            for c in candidates:
                trial = list(best)
                trial[b] = c
                ms = _time_call(call(trial), reps)
                trace.append({"blocks": trial, "ms": ms})
                if ms < best_ms:
                    best_ms, best = ms, trial
    cache = load_cache(path)
    for b in range(3):
        cache[cache_key(b, desc.prec, desc.t_max)] = {"blocks": best[b], "ms": best_ms}
    save_cache(cache, path)
    return best, best_ms, default_ms, trace
