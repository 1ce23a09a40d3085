"""Secondary benchmark workloads of bench.py (``--workload``): joint channel
estimation and detection with 16 antennas and 16 data slots plus a pilot
(262,144 blocks, t_max = 20), and coherent 32x8 QPSK detection (1,000
vectors, one channel each, t_max = 10).  Same protocol as the headline:
inputs resident in HBM, warm-up, timed launches bracketed by HIP events on
the launch stream, paired BER against the FP64 oracle on a sample.
"""
from __future__ import annotations

import os
import time

import numpy as np

import sim

PEAK_FP32 = 157.3


def loop_flops(N, t_max):
    s2 = N * (N + 1) * (2 * N + 1) // 6
    return t_max * (2 * s2 + 3 * N * (N + 1) // 2 + 2 * N)


def own_build_flops(B, U, N, mod):
    """T assembly for one vector with its own channel: complex Gram
    (Hermitian, 8B U(U+1)/2), matched filter 8BU, ||y||^2 4B, preconditioning
    scaling ~2N^2 (the BPSK real parts halve the Gram and matched filter)."""
    f = 8 * B * U * (U + 1) // 2 + 8 * B * U
    if mod == 1:
        f //= 2
    return f + 4 * B + 2 * N * N


def _oracle_sample(kind, d, idx, mod, t_max, alpha):
    """Oracle decisions for the sampled vectors (single process: the sample
    is bounded to a few seconds of CPU work)."""
    import oracle
    if kind == "jed":
        return oracle.detect_jed(d["Y"][idx], d["s0"][idx], mod, alpha=alpha, t_max=t_max)["sbar"]
    Hv = np.repeat(d["H"], d["y_per_H"], axis=0)[idx]
    return oracle.detect_coherent(Hv, d["y"][idx], mod, alpha=alpha, t_max=t_max)["sbar"]


def _time(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def run_workload(args):
    import torch
    import paper_1609_01797_amd as taser
    if args.workload == "jed16x16":
        kind, B, U, mod, V, t_max, alpha = "jed", 16, 16, 2, 262144, 20, 0.5
        snrs, snr_timed, sample = [0.0, 2.0, 4.0, 6.0, 8.0, 10.0, 12.0], 6.0, 16384
        metric = "detected blocks/s @SIMO JED 16 antennas, 16+1 QPSK slots, t_max=20 (262,144 blocks)"
    else:
        kind, B, U, mod, V, t_max, alpha = "coh", 32, 8, 2, 1000, 10, 0.5
        snrs, snr_timed, sample = [0.0, 2.0, 4.0, 6.0, 8.0, 10.0], 10.0, 1000
        metric = "detected vectors/s @32x8 QPSK t_max=10 (1,000 vectors, one channel each)"
    N = 2 * U + 1 if mod == 2 else U + 1
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(V, size=min(sample, V), replace=False))
    precs = (("bf16", 1), ("fp32", 0), ("fp16", 2))
    res = {"paths": {}, "ber": {p: [] for p, _ in precs}, "ber_fp64_sample": [], "ber_sample": {p: [] for p, _ in precs}}
    cpu_seconds = 0.0
    for snr in snrs:
        if kind == "jed":
            d = sim.gen_jed(B, U, mod, V, snr, sim.seed_for(5, snr_index=int(snr)))
            truth = np.concatenate([d["s"][:, 1:].real, d["s"][:, 1:].imag], axis=1).astype(np.int8)
            ins = (None, torch.from_numpy(d["Y"]).to(dev), torch.from_numpy(d["s0"]).to(dev))
        else:
            d = sim.gen_mimo(B, U, mod, V, 1, snr, sim.seed_for(1, snr_index=int(snr)))
            truth = np.concatenate([d["s"].real, d["s"].imag], axis=1).astype(np.int8)
            ins = (torch.from_numpy(d["H"]).to(dev), torch.from_numpy(d["y"]).to(dev), None)
        t0 = time.perf_counter()
        ref = _oracle_sample(kind, d, idx, mod, t_max, alpha)
        cpu_seconds += time.perf_counter() - t0
        res["ber_fp64_sample"].append(float(np.mean(ref != truth[idx])))
        for name, prec in precs:
            desc = taser.make_desc(V, B, U, mod, mode=taser.JED if kind == "jed" else taser.COHERENT,
                                   prec=prec, t_max=t_max, alpha=alpha)
            out = {}
            fn = lambda: taser.run(desc, ins[0], ins[1], ins[2], out=out)  # noqa: E731
            fn()
            sb = out["sbar"].cpu().numpy()
            res["ber"][name].append(float(np.mean(sb != truth)))
            res["ber_sample"][name].append(float(np.mean(sb[idx] != truth[idx])))
            if snr == snr_timed:
                ms = _time(fn, args.steps, args.warmup, stream)
                res["paths"][name] = {"kernel_ms": ms, "per_s": V / (ms * 1e-3)}
        del d, ins
        torch.cuda.empty_cache()
    fl = loop_flops(N, t_max) + own_build_flops(B, U, N, mod)
    fp32 = res["paths"]["fp32"]
    fp32["tflops"] = fl * V / (fp32["kernel_ms"] * 1e-3) / 1e12
    fp32["frac_fp32_peak"] = fp32["tflops"] / PEAK_FP32
    head = res["paths"]["bf16"]
    return {"metric": metric, "value": head["per_s"], "unit": "blocks/s" if kind == "jed" else "vectors/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["kernel_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic",
            "config": {"workload": args.workload, "B": B, "K_or_U": U, "modulation": "QPSK", "N": N,
                       "vectors": V, "t_max": t_max, "alpha": alpha, "snr_db_timed": snr_timed,
                       "tau": "spectral"},
            "roofline_fp32": {"bound": "mfma", "kernel": "fused_vec", "achieved": fp32["tflops"],
                              "peak": PEAK_FP32, "unit": "TFLOP/s", "frac": fp32["frac_fp32_peak"],
                              "flops_per_vector": fl},
            "cpu_baseline": {"value": len(idx) * len(snrs) / cpu_seconds, "unit": "vectors/s", "cores": 1,
                             "kind": "oracle", "sample": f"{len(idx)} sampled vectors per SNR point x "
                             f"{len(snrs)} points, one process"},
            "accuracy": {"snr_db": snrs, "ber": res["ber"], "sample_size": int(len(idx)),
                         "ber_fp64_sample": res["ber_fp64_sample"], "ber_gpu_sample": res["ber_sample"]},
            "paths": res["paths"]}
