"""Mixed-size batches in one call (taser_run_mixed): parity with the FP64
oracle per vector, HIP-graph capture and replay, launch configurations,
and vectors outside the fused kernels."""
import numpy as np
import pytest

import oracle
import sim
from parity import assert_decisions, L_REL_TOL

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _inputs(d):
    return (_cuda(d["B"]), _cuda(d["U"]), _cuda(d["mod"]), _cuda(d["H_off"]), _cuda(d["y_off"]),
            _cuda(d["H_flat"]), _cuda(d["y_flat"]))


def _oracle_mixed(d, alpha, t_max):
    """Oracle per size class; returns per-vector sbar (padded to 64), margin."""
    V = len(d["cls"])
    sbar = np.ones((V, 64), dtype=np.int8)
    margin = np.zeros((V, 64))
    tau = np.zeros(V)
    for c in np.unique(d["cls"]):
        idx = np.nonzero(d["cls"] == c)[0]
        B, U, mod = int(d["B"][idx[0]]), int(d["U"][idx[0]]), int(d["mod"][idx[0]])
        H = np.stack([d["H_flat"][d["H_off"][v]:d["H_off"][v] + B * U].reshape(B, U) for v in idx])
        y = np.stack([d["y_flat"][d["y_off"][v]:d["y_off"][v] + B] for v in idx])
        r = oracle.detect_coherent(H, y, mod, alpha=alpha, t_max=t_max)
        n = oracle.problem_size(U, mod) - 1
        sbar[idx, :n] = r["sbar"]
        margin[idx, :n] = r["margin"]
        tau[idx] = r["tau"]
    return sbar, margin, tau


@pytest.fixture(scope="module")
def mixed_case():
    d = sim.gen_mixed(900, 12.0, sim.seed_for(3, snr_index=6))
    return d, _oracle_mixed(d, 0.5, 10)


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp32", "bf16", "fp16"])
def test_mixed_parity(gpu_lib, mixed_case, prec):
    import torch
    d, (sbar_ref, margin_ref, tau_ref) = mixed_case
    V = len(d["cls"])
    mtol = {0: 1e-4, 1: 10 * 2.0 ** -8, 2: 10 * 2.0 ** -11}[prec]
    desc = gpu_lib.make_desc(V, 1, 1, 2, prec=prec, tau_mode=gpu_lib.TAU_GIVEN, t_max=10)
    res = gpu_lib.run_mixed(desc, *_inputs(d), tau=_cuda(tau_ref.astype(np.float32)), want_margin=True)
    torch.cuda.synchronize()
    sb, mg = res["sbar"].cpu().numpy(), res["margin"].cpu().numpy()
    assert np.all(res["status"].cpu().numpy() == 0)
    for v in range(V):
        n = oracle.problem_size(int(d["U"][v]), int(d["mod"][v])) - 1
        assert_decisions(sb[v:v + 1, :n], sbar_ref[v:v + 1, :n], margin_ref[v:v + 1, :n], tol=mtol)
    # margins carry L~'s last row: float32 within the L~ tolerance scale
    if prec == 0:
        for v in range(V):
            n = oracle.problem_size(int(d["U"][v]), int(d["mod"][v])) - 1
            np.testing.assert_allclose(mg[v, :n], margin_ref[v, :n], atol=20 * L_REL_TOL)
    # spectral step size on the GPU
    desc2 = gpu_lib.make_desc(V, 1, 1, 2, prec=prec, t_max=10, alpha=0.5)
    res2 = gpu_lib.run_mixed(desc2, *_inputs(d))
    sb2 = res2["sbar"].cpu().numpy()
    for v in range(V):
        n = oracle.problem_size(int(d["U"][v]), int(d["mod"][v])) - 1
        assert_decisions(sb2[v:v + 1, :n], sbar_ref[v:v + 1, :n], margin_ref[v:v + 1, :n], tol=mtol)


def test_mixed_launch_configs_agree(gpu_lib, mixed_case):
    import torch
    d, _ = mixed_case
    V = len(d["cls"])
    desc = gpu_lib.make_desc(V, 1, 1, 2, t_max=10, alpha=0.5)
    ins = _inputs(d)
    base = gpu_lib.run_mixed(desc, *ins, want_margin=True)
    base = {k: v.clone() for k, v in base.items()}
    for blocks in ([1, 1, 1], [7, 3, 2], [0, 5, 0], [4096, 4096, 4096]):
        r = gpu_lib.run_mixed(desc, *ins, want_margin=True, blocks=blocks)
        torch.cuda.synchronize()
        for k in ("sbar", "margin", "status"):
            assert torch.equal(r[k], base[k]), (blocks, k)
    # the alternative register budgets, the single launch over one work
    # queue and the bucket kernels on three streams run the same arithmetic
    for waves, single, conc in (([1, 1, 1], False, False), ([1, 0, 1], False, False),
                                ([0, 0, 0], True, False), ([1, 1, 1], True, False),
                                ([0, 0, 0], False, True), ([1, 0, 1], False, True)):
        r = gpu_lib.run_mixed(desc, *ins, want_margin=True, waves=waves, single=single, concurrent=conc)
        torch.cuda.synchronize()
        for k in ("sbar", "margin", "status"):
            assert torch.equal(r[k], base[k]), (waves, single, conc, k)
    # a persistent grid on the side streams
    r = gpu_lib.run_mixed(desc, *ins, want_margin=True, blocks=[7, 3, 2], concurrent=True)
    torch.cuda.synchronize()
    for k in ("sbar", "margin", "status"):
        assert torch.equal(r[k], base[k]), ("blocks concurrent", k)


@pytest.mark.parametrize("concurrent", [False, True])
def test_mixed_graph_capture_replay(gpu_lib, mixed_case, concurrent):
    """The mixed call captured into a HIP graph gives the eager result on
    every replay, with unrelated eager work and synchronisation in between
    (with concurrent buckets the capture forks into the library's side
    streams and joins back)."""
    import torch
    d, _ = mixed_case
    V = len(d["cls"])
    desc = gpu_lib.make_desc(V, 1, 1, 2, prec=1, t_max=10, alpha=0.5)
    ins = _inputs(d)
    eager = gpu_lib.run_mixed(desc, *ins, want_margin=True)
    eager = {k: v.clone() for k, v in eager.items()}
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    out = {"sbar": torch.empty_like(eager["sbar"]), "status": torch.empty_like(eager["status"]),
           "margin": torch.empty_like(eager["margin"])}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        # warm up on the side stream (this also creates the library's side
        # streams, which cannot be created while a stream is being captured)
        gpu_lib.run_mixed(desc, *ins, want_margin=True, out=out, ws=ws, concurrent=concurrent)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gpu_lib.run_mixed(desc, *ins, want_margin=True, out=out, ws=ws, concurrent=concurrent)
    for rep in range(4):
        for k in out:
            out[k].zero_()
        junk = torch.randn(4096, device="cuda").sum()   # unrelated eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in out:
            assert torch.equal(out[k], eager[k]), (rep, k)
        del junk


def test_mixed_unsupported_sizes(gpu_lib):
    import torch
    classes = ((32, 8, 2), (48, 40, 2))            # the second has U > 32
    d = sim.gen_mixed(40, 10.0, 99, classes=classes)
    V = 40
    desc = gpu_lib.make_desc(V, 1, 1, 2, t_max=5, alpha=0.5)
    res = gpu_lib.run_mixed(desc, *_inputs(d))
    torch.cuda.synchronize()
    st = res["status"].cpu().numpy()
    big = d["U"] == 40
    assert np.all(st[big] == gpu_lib.VEC_UNSUPPORTED)
    assert np.all(st[~big] == 0)
    sb = res["sbar"].cpu().numpy()
    assert np.all(sb[big][:, :64] == 1)          # N - 1 = 80 > stride: the whole row is +1
    assert np.all(sb[~big][:, 16:] == 0)         # padding past N - 1 = 16 is 0


def _alpha_star(name):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "alpha_star.json")
    return float(json.load(open(path))["workloads"][name]["alpha_star"])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16"])
def test_mixed_full_batch_bench_configuration(gpu_lib, prec):
    """The benchmark's mixed launch: 100,000 vectors over the six classes,
    SNR 12 dB, t_max = 10, the swept alpha, tau spectral, default grid.
    Decisions are checked against the oracle on 300 sampled vectors of each
    class; the padding of every row is zero."""
    import torch
    alpha = _alpha_star("mixed")
    V = 100000
    d = sim.gen_mixed(V, 12.0, sim.seed_for(3, snr_index=6))
    desc = gpu_lib.make_desc(V, 1, 1, 2, prec=prec, t_max=10, alpha=alpha)
    res = gpu_lib.run_mixed(desc, *_inputs(d), want_margin=False)
    torch.cuda.synchronize()
    sb, st = res["sbar"].cpu().numpy(), res["status"].cpu().numpy()
    assert np.all(st == 0)
    nm1 = np.where(d["mod"] == 2, 2 * d["U"], d["U"])
    assert np.all(sb[np.arange(64)[None, :] >= nm1[:, None]] == 0)
    mtol = {0: 1e-4, 1: 10 * 2.0 ** -8}[prec]
    rng = np.random.default_rng(11)
    for c in range(len(sim.MIXED_CLASSES)):
        idx = np.sort(rng.choice(np.nonzero(d["cls"] == c)[0], size=300, replace=False))
        B, U, mod = int(d["B"][idx[0]]), int(d["U"][idx[0]]), int(d["mod"][idx[0]])
        H = np.stack([d["H_flat"][d["H_off"][v]:d["H_off"][v] + B * U].reshape(B, U) for v in idx])
        y = np.stack([d["y_flat"][d["y_off"][v]:d["y_off"][v] + B] for v in idx])
        ref = oracle.detect_coherent(H, y, mod, alpha=alpha, t_max=10)
        n = oracle.problem_size(U, mod) - 1
        assert_decisions(sb[idx, :n], ref["sbar"], ref["margin"], tol=mtol)


def test_mixed_concurrent_from_two_host_threads(gpu_lib, mixed_case):
    """Two host threads call the concurrent form at the same time, each on its
    own stream: they share the library's side streams and events (the
    enqueue is serialised), and every call gives the sequential result."""
    import threading

    import torch
    d, _ = mixed_case
    V = len(d["cls"])
    desc = gpu_lib.make_desc(V, 1, 1, 2, prec=1, t_max=10, alpha=0.5)
    ins = _inputs(d)
    base = gpu_lib.run_mixed(desc, *ins, want_margin=True)
    base = {k: v.clone() for k, v in base.items()}
    torch.cuda.synchronize()
    results, errors = [[], []], []

    def worker(slot):
        try:
            stream = torch.cuda.Stream()
            ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
            with torch.cuda.stream(stream):
                for _ in range(4):
                    r = gpu_lib.run_mixed(desc, *ins, want_margin=True, concurrent=True, ws=ws)
                    results[slot].append({k: v.clone() for k, v in r.items()})
            stream.synchronize()
        except Exception as e:   # surfaced by the assertion below
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for slot in range(2):
        assert len(results[slot]) == 4
        for r in results[slot]:
            for k in ("sbar", "margin", "status"):
                assert torch.equal(r[k], base[k]), (slot, k)
