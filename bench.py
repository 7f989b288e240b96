"""Throughput of damped log-domain loopy BP on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload potts512]

A step is one whole solve on a graph already resident in HBM: reset the
messages, run the iterations (variable phase + factor phase, damping and
normalisation fused), then read out normalised beliefs and the MAP into
device buffers.  K steps are timed between device synchronisations.

Metric: edge-state message updates per second = ES * iters * K / seconds.
The JSON line also carries the roofline of the dominant kernel (the factor
phase), timed live with HIP events on the library's stream, and the FP64
oracle timed on the host's cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
LLC_BYTES = 256 << 20  # MI355X last-level (Infinity) cache

WORKLOADS = {
    # name: (builder, iters, damping, temperature, description)
    "potts512": (lambda W: W.potts_grid(512, 5, seed=2), 200, 0.5, 1.0,
                 "Potts grid 512x512, 5 states, 4-neighbour pairwise factors, sum-product T=1, "
                 "damping 0.5, 200 iterations, FP32"),
    "potts2048": (lambda W: W.potts_grid(2048, 5, seed=2), 200, 0.5, 1.0,
                  "Potts grid 2048x2048, 5 states (scale-up beyond the 256 MB last-level cache), "
                  "sum-product T=1, damping 0.5, 200 iterations, FP32"),
    "ising32": (lambda W: W.ising_grid(32, seed=1), 100, 0.5, 0.0,
                "Ising grid 32x32, max-product, damping 0.5, 100 iterations, FP32"),
    "rbm": (lambda W: W.rbm(784, 500, seed=3), 200, 0.5, 0.0,
            "RBM 784 visible x 500 hidden, all 392000 pairwise factors, max-product, damping 0.5, "
            "200 iterations, FP32"),
    "rbm_t005": (lambda W: W.rbm(784, 500, seed=3), 200, 0.5, 0.05,
                 "RBM 784 visible x 500 hidden, all 392000 pairwise factors, sum-product at T=0.05, "
                 "damping 0.5, 200 iterations, FP32"),
    "triplet256": (lambda W: W.triplet_grid(256, 3, seed=12), 100, 0.5, 1.0,
                   "three-way factors on a 256x256 grid (every three consecutive variables along rows and "
                   "columns), 3 states, dense 27-entry tables, sum-product T=1, damping 0.5, 100 iterations, FP32"),
    "deconv": (lambda W: W.deconv(seed=4), 1000, 0.5, 0.0,
               "binary deconvolution with OR/AND factors, 5 templates 6x6, 32x32 image, "
               "max-product, damping 0.5, 1000 iterations, FP32"),
}


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "lbp_internal.h"):
        with open(os.path.join(ROOT, "paper_2202_04110_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def byte_model(spec, iters):
    """Algorithmic bytes (index arrays excluded).

    A message is one row per state, except a two-state message, which is one
    number (its rows are normalised, so m1 - m0 determines both): MS stored
    message floats, ES - (two-state edges).
    factor phase per launch: read potentials 4*Tn, read messages 4*MS, read
    beliefs 4*VS (each unique belief once), write messages 4*MS.
    variable phase per launch: read messages 4*MS, evidence 4*VS, write beliefs 4*VS.
    """
    ES, VS, Tn = spec.num_edge_states, spec.num_var_states, spec.num_logpots
    two = int(np.count_nonzero(np.asarray(spec.var_num_states)[np.asarray(spec.edge_var)] == 2))
    MS = ES - two
    factor = 4 * Tn + 8 * MS + 4 * VS
    var = 4 * MS + 8 * VS
    return {"factor_bytes": factor, "variable_bytes": var, "iter_bytes": factor + var,
            "floor_bytes": 8 * MS + 4 * Tn + 4 * VS, "message_floats": MS}


def measured_traffic(workload, kernel, shape):
    """Bytes per launch that L2 exchanged with the memory side for `kernel`
    ("fused", "factor" or "variable"), from the committed rocprofv3 counter
    summary, scaled by the copy calibration; None unless the summary was taken
    on the current kernel sources with the same launch shape."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    k = t.get("kernels", {}).get(kernel)
    if t.get("kernel_src_sha") != kernel_source_sha() or not k:
        return None
    if [k.get("wpb"), k.get("swizzle")] != list(shape):
        return None
    return k.get("bytes_per_launch")


def plain_copy_gbps(mib=1024, reps=10):
    """Read + write GB/s of a plain device-to-device copy of `mib` MiB (the
    runtime's copy kernel), timed with HIP events: the bandwidth an ordinary
    streaming kernel reaches on this machine, beside the nominal peak."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.empty(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def stream_probes(ctx, mib=1024, blocks=(512, 1024, 2048, 4096), reps=5):
    """The library's plain streaming kernels (lbp_bandwidth_probe: float4,
    grid-stride) over `mib` MiB, the best of a few grid sizes per kind: the
    bandwidth an ordinary kernel reaches on this device, per read/write mix."""
    import torch

    n = mib * (1 << 20)
    a = torch.zeros(n // 4, dtype=torch.float32, device="cuda")
    b = torch.zeros(n // 4, dtype=torch.float32, device="cuda")
    out = {"bytes": n, "blocks_tried": list(blocks)}
    for kind, name, moved in ((0, "read_gbps", 1.0), (1, "copy_gbps", 2.0), (2, "write_gbps", 1.0),
                              (3, "mix5r1w_gbps", 1.2)):
        nb = n if kind != 3 else (n // 80) * 80
        best = max(moved * nb / (ctx.bandwidth_probe(kind, a, b, nb, bl, reps) * 1e-3) / 1e9 for bl in blocks)
        out[name] = best
    del a, b
    torch.cuda.empty_cache()
    return out


def cpu_baseline(spec, iters_full, damping, temperature, budget_s=12.0):
    """The FP64 oracle on the host's cores, timed on a bounded number of
    iterations of the same graph; scaled to edge-state updates per second."""
    from oracle import OracleGraph

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    og = OracleGraph(spec)
    og.run(1, damping, temperature, threads=cores)
    t1 = og.last_seconds
    iters = int(max(1, min(iters_full, budget_s / max(t1, 1e-6))))
    m = og.run(iters, damping, temperature, threads=cores)
    dt = og.last_seconds
    del m
    # the same oracle on one core, on a shorter sample
    iters1 = int(max(1, min(iters_full, 0.3 * budget_s / max(t1 * cores, 1e-6))))
    m = og.run(iters1, damping, temperature, threads=1)
    dt1 = og.last_seconds
    del m
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": spec.num_edge_states * iters / dt, "unit": "edge-state updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d of %d iterations of the same graph, FP64, OpenMP over variables and factors, "
                      "%.2f s" % (iters, iters_full, dt),
            "one_core": {"value": spec.num_edge_states * iters1 / dt1, "sample": "%d iterations, %.2f s" % (iters1, dt1)},
            "host_cpu": model, "host_cpus_visible": os.cpu_count()}


def serving_leg(lbp, W, ctx, n, budgets_mb, seed=5, steps=10, slots=64):
    """Served stream: n Potts requests (side log-uniform 16..256, 2..8
    states, sum-product T=1, damping 0.5, 50 iterations; 10% carry a backward
    pass with checkpoints every 10), per HBM budget.  Capacity R is measured
    with every request arriving at once (after one untimed burst that warms
    the pinned result pool, as a long-running server's would be); then
    Poisson arrivals at 0.5R, 0.8R and 1.0R give p50/p99 latency (completion
    minus scheduled arrival).
    "burst, early exit": the burst again with the forward requests stopping
    once their residual (checked every 5 iterations) is below 1e-3."""
    from paper_2202_04110_amd.serving import run_stream

    reqs = W.served_requests(n, seed=seed, backward_count=max(1, n // 10))
    specs = [W.request_graph(r) for r in reqs]
    gqs = [W.request_loss_coeffs(r) if r["backward"] else None for r in reqs]
    out = {"requests": n, "iters": 50, "backward_requests": sum(g is not None for g in gqs),
           "max_slots": slots, "steps_per_round": steps,
           "edge_states_mean": float(np.mean([s.num_edge_states for s in specs])), "budgets": {},
           "warmup": "one untimed burst of the same requests first (fills the process-wide pinned result pool)"}
    srv = lbp.Server(ctx, budget_bytes=budgets_mb[0] << 20, max_slots=slots, steps_per_round=steps)
    run_stream(srv, specs, np.zeros(n), 50, 0.5, 1.0, grad_qs=gqs, ckpt_every=10)
    srv.close()
    for budget_mb in budgets_mb:
        runs = {}
        for label, frac in (("burst", None), ("0.5R", 0.5), ("0.8R", 0.8), ("1.0R", 1.0),
                            ("burst, early exit", None)):
            srv = lbp.Server(ctx, budget_bytes=budget_mb << 20, max_slots=slots, steps_per_round=steps)
            if frac is None:
                arr = np.zeros(n)
            else:
                arr = W.poisson_arrivals(n, qps=frac * runs["burst"]["requests_per_s"], seed=seed)
            tol = 1e-3 if "early" in label else None
            _, summ = run_stream(srv, specs, arr, 50, 0.5, 1.0, grad_qs=gqs, ckpt_every=10, tol=tol, check_every=5)
            srv.close()
            st = summ.pop("stats")
            for k in ("max_resident", "rounds", "busy_us", "round_us", "prep_us", "prep_threads", "admit_us",
                      "launch_us", "finish_us"):
                summ[k] = st[k]
            runs[label] = summ
            print("serving budget %d MB %s: %.0f req/s p50 %.2f ms p99 %.2f ms, %.1f iterations per request" % (
                budget_mb, label, summ["requests_per_s"] or 0, 1e3 * (summ["p50_s"] or 0),
                1e3 * (summ["p99_s"] or 0), summ["iters_mean"] or 0), file=sys.stderr, flush=True)
        out["budgets"]["%d MB" % budget_mb] = runs
    return out


def gradient_leg(lbp, W, ctx, reps=10, side=64, states=6, iters=50, every=10):
    """Cost of a gradient: a Potts side x side grid with `states` states
    (sum-product T=1, damping 0.5, `iters` iterations) solved forward only,
    then recorded with checkpoints every `every` iterations and swept back
    for dL/dphi and dL/dtheta of a fixed linear loss on the beliefs."""
    import torch

    spec = W.potts_grid(side, states, seed=7)
    g = lbp.Graph(ctx, spec)
    gq = torch.from_numpy(np.random.default_rng(7).standard_normal(g.VS).astype(np.float32)).cuda()
    gphi = torch.empty(len(spec.log_potentials), device="cuda", dtype=torch.float32)
    gth = torch.empty(g.VS, device="cuda", dtype=torch.float32)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    def fwd():
        g.reset_messages()
        g.run_bp(iters, 0.5, 1.0)

    def rec():
        g.reset_messages()
        g.run_bp_record(iters, 0.5, 1.0, every)

    def both():
        rec()
        g.backward(gq, gphi, gth)

    t_f, t_r, t_b = timed(fwd), timed(rec), timed(both)
    g.free()
    return {"graph": "Potts %dx%d, %d states, %d iterations, checkpoints every %d" % (side, side, states, iters, every),
            "edge_states": spec.num_edge_states, "forward_ms": t_f, "record_ms": t_r,
            "record_plus_backward_ms": t_b, "backward_over_forward": (t_b - t_r) / t_f}


def sampling_leg(lbp, W, ctx, S, iters=1000, reps=3):
    """Perturb-and-MAP on the deconvolution workload: S samples (Gumbel(0,1)
    noise on the evidence, max-product, damping 0.5, `iters` iterations)
    in shared launches, against one plain solve of the same graph."""
    import torch

    spec = W.deconv(seed=4)
    g = lbp.Graph(ctx, spec)
    gen = torch.Generator(device="cuda").manual_seed(11)
    u = torch.rand((S, g.VS), device="cuda", generator=gen).clamp_(1e-12, 1 - 1e-12)
    noise = (-torch.log(-torch.log(u))).contiguous()
    sp = lbp.Sampler(g, S)
    mp = torch.empty((S, g.V), device="cuda", dtype=torch.int32)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def one():
        g.reset_messages()
        g.run_bp(iters, 0.5, 0.0)
        g.decode_map(out=mp[0])

    t1 = timed(one)
    ts = timed(lambda: sp.run(iters, 0.5, 0.0, noise, map_out=mp))
    sp.free()
    g.free()
    return {"graph": "binary deconvolution (OR/AND factors), max-product, damping 0.5, %d iterations" % iters,
            "samples": S, "edge_states": spec.num_edge_states, "single_solve_ms": t1 * 1e3,
            "sample_batch_ms": ts * 1e3, "samples_per_s": S / ts,
            "edge_state_updates_per_s": spec.num_edge_states * iters * S / ts,
            "speedup_over_sequential": S * t1 / ts}


def batch_leg(lbp, W, ctx, n, iters=50, reps=5, seed=5):
    """n graphs of the served mix (Potts, side 16..256 log-uniform, 2..8
    states, sum-product T=1, damping 0.5, `iters` iterations) advanced
    together in one batch: two-phase iterations, fused iterations, after
    lbp_batch_autotune, and the same graphs solved one after another."""
    import torch

    reqs = W.served_requests(n, seed=seed, backward_count=0)
    specs = [W.request_graph(r) for r in reqs]
    gs = [lbp.Graph(ctx, s) for s in specs]
    b = lbp.Batch(ctx, gs)
    es = sum(int(s.num_edge_states) for s in specs)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def lone():
        for g in gs:
            g.run_bp(iters, 0.5, 1.0)

    t_lone = timed(lone)
    t_two = timed(lambda: b.run_bp(iters, 0.5, 1.0))
    b.use_fused(True)
    t_fused = timed(lambda: b.run_bp(iters, 0.5, 1.0))
    tuned_fused = b.autotune(0.5, 1.0, reps=10)
    t_tuned = timed(lambda: b.run_bp(iters, 0.5, 1.0))
    b.free()
    for g in gs:
        g.free()
    return {"graphs": n, "iters": iters, "edge_states": es,
            "one_after_another_ms": t_lone * 1e3, "batch_two_phase_ms": t_two * 1e3, "batch_fused_ms": t_fused * 1e3,
            "batch_autotuned_ms": t_tuned * 1e3, "autotune_chose_fused": tuned_fused,
            "edge_state_updates_per_s": {"one_after_another": es * iters / t_lone, "batch_two_phase": es * iters / t_two,
                                         "batch_fused": es * iters / t_fused, "batch_autotuned": es * iters / t_tuned}}


def scaleup_leg(lbp, W, ctx, tune, reps=50, solves=3):
    """The HBM-bound case: Potts 2048x2048x5 (1.6 GB of floor bytes per
    iteration, beyond the 256 MB last-level cache), sum-product T=1, damping
    0.5, 200 iterations, in the shipped launch shapes.  Roofline of the fused
    iteration launch (floor bytes over its HIP-event launch time) and whole
    solves timed between device synchronisations."""
    import torch

    spec = W.potts_grid(2048, 5, seed=2)
    iters, d, T = 200, 0.5, 1.0
    g = lbp.Graph(ctx, spec)
    tuned = tune.apply_or_tune(g, d, T)
    bm = byte_model(spec, iters)
    ES = spec.num_edge_states
    del spec
    q = torch.empty(g.VS, device="cuda", dtype=torch.float32)
    mp = torch.empty(g.V, device="cuda", dtype=torch.int32)

    def solve():
        g.reset_messages()
        g.run_bp(iters, d, T)
        g.get_beliefs(out=q)
        g.decode_map(out=mp)

    solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(solves):
        solve()
    torch.cuda.synchronize()
    ms_solve = (time.perf_counter() - t0) * 1e3 / solves
    g.status()
    fl = [l for l in g.launches() if l["phase"] == 1]
    out = {"workload": WORKLOADS["potts2048"][4], "edge_states": ES, "ms_per_solve": ms_solve,
           "edge_state_updates_per_s": ES * iters / (ms_solve * 1e-3), "fused_iterations": g.fused_in_use,
           "tune_source": tuned["source"]}
    if g.fused_in_use:
        kms = g.time_phase(3, reps, d, T)
        kbytes = bm["floor_bytes"]
        shape = (fl[0]["fused_wpb"], fl[0]["fused_variant"])
        kernel, tkey = "fused iteration (dense pairwise factors, beliefs recomputed)", "fused"
    else:
        kms = g.time_phase(1, reps, d, T)
        kbytes = bm["factor_bytes"]
        shape = (fl[0]["wpb"], fl[0]["swizzle"])
        kernel, tkey = "factor phase", "factor"
    achieved = kbytes / (kms * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": measured_traffic("potts2048", tkey, shape), "kernel": kernel,
                       "algorithmic_bytes_per_launch": kbytes, "avg_launch_ms": kms,
                       "launch_shape": list(shape)}
    g.free()
    torch.cuda.empty_cache()
    return out


def small_graphs_leg(lbp, W, ctx, tune, solves=5, reps=200):
    """The paper's small workloads in the shipped launch shapes: the RBM
    784x500 (200 max-product iterations) and the deconvolution graph (1000),
    each timed as whole solves (message reset, iterations, beliefs and MAP
    into device buffers) between device synchronisations, plus the RBM's
    variable phase in place against its algorithmic bytes."""
    import torch

    out = {}
    for name in ("rbm", "deconv"):
        make, iters, d, T, desc = WORKLOADS[name]
        spec = make(W)
        g = lbp.Graph(ctx, spec)
        tuned = tune.apply_or_tune(g, d, T)
        bm = byte_model(spec, iters)
        ES = spec.num_edge_states
        q = torch.empty(g.VS, device="cuda", dtype=torch.float32)
        mp = torch.empty(g.V, device="cuda", dtype=torch.int32)

        def solve():
            g.reset_messages()
            g.run_bp(iters, d, T)
            g.get_beliefs(out=q)
            g.decode_map(out=mp)

        solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(solves):
            solve()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / solves
        g.status()
        r = {"workload": desc, "ms_per_solve": ms, "us_per_iteration": 1e3 * ms / iters,
             "edge_state_updates_per_s": ES * iters / (ms * 1e-3), "tune_source": tuned["source"],
             "launch_shapes": [[l["phase"], l["wpb"], l["swizzle"]] for l in g.launches()]}
        if name == "rbm":
            tv = g.time_phase(0, reps, d, T)
            ach = bm["variable_bytes"] / (tv * 1e-3) / 1e9
            r["variable_phase"] = {"avg_launch_ms": tv, "algorithmic_bytes_per_launch": bm["variable_bytes"],
                                   "achieved_gbps": ach, "frac": ach / HBM_PEAK_GBS}
        out[name] = r
        g.free()
        del spec
    torch.cuda.empty_cache()
    return out


def paper_rbm_leg(lbp, W, ctx, runs=10):
    """The paper's timing protocol on MAP inference: fully connected binary
    RBMs of 40, 60, ..., 200 units (half visible, half hidden), max-product,
    200 iterations, damping 0.5, each time the mean of `runs` solves.  A solve
    is reset messages + 200 iterations + MAP decode copied to the host, with
    the graph resident in HBM; the second figure also uploads the graph (and
    captures its loop) every time."""
    import torch

    out = {}
    for units in range(40, 201, 20):
        spec = W.rbm(units // 2, units // 2, seed=units)
        g = lbp.Graph(ctx, spec)
        g.run_bp(200, 0.5, 0.0)
        g.decode_map()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(runs):
            g.reset_messages()
            g.run_bp(200, 0.5, 0.0)
            g.decode_map()
        t_res = (time.perf_counter() - t0) / runs
        g.free()
        t0 = time.perf_counter()
        for _ in range(runs):
            h = lbp.Graph(ctx, spec)
            h.run_bp(200, 0.5, 0.0)
            h.decode_map()
            h.free()
        t_up = (time.perf_counter() - t0) / runs
        es = int(spec.num_edge_states)
        out[str(units)] = {"edge_states": es, "solve_ms": t_res * 1e3, "upload_and_solve_ms": t_up * 1e3,
                           "edge_state_updates_per_s": es * 200 / t_res}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="potts512", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phase-reps", type=int, default=200)
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--serving", type=int, default=512, metavar="N",
                    help="also run the served stream with N requests (0: skip)")
    ap.add_argument("--serving-budget-mb", default="512,2048",
                    help="comma-separated HBM budgets of the served stream, in MiB")
    ap.add_argument("--serving-steps", type=int, default=10,
                    help="iterations per server round (requests join and leave at round boundaries)")
    ap.add_argument("--serving-slots", type=int, default=64, help="most requests resident at once")
    ap.add_argument("--samples", type=int, default=0, metavar="S",
                    help="also time S perturb-and-MAP samples of the deconvolution graph in shared launches")
    ap.add_argument("--batch", type=int, default=64, metavar="N",
                    help="batch leg: N served-mix graphs in one batch, two-phase and fused iterations (0: skip)")
    ap.add_argument("--paper-rbm", action="store_true",
                    help="the paper's MAP timing protocol: RBMs of 40..200 units, 200 max-product iterations")
    ap.add_argument("--no-gradient", action="store_true",
                    help="skip timing a recorded solve plus its reverse sweep against the forward solve")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the RBM 784x500 and deconvolution per-iteration leg")
    ap.add_argument("--no-scaleup", action="store_true",
                    help="skip the Potts 2048x2048 roofline (the HBM-bound case)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed workload and its roofline (no serving, batch, gradient, scale-up, "
                         "small-graph or CPU baseline legs), e.g. under a profiler")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes 5 times (the reference "
                         "kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.headline_only:
        args.serving = args.batch = args.samples = 0
        args.no_gradient = args.no_scaleup = args.no_cpu_baseline = args.no_small = True
        args.paper_rbm = False
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                          "launches": 5}))
        return

    from paper_2202_04110_amd import lbp, tune
    from paper_2202_04110_amd import workloads as W

    build, iters, d, T, desc = WORKLOADS[args.workload]
    spec = build(W)
    torch.cuda.set_device(0)
    ctx = lbp.Context(0)
    g = lbp.Graph(ctx, spec)
    tuned = None
    if not args.no_tune:
        tuned = tune.apply_or_tune(g, d, T)
    q = torch.empty(g.VS, device="cuda", dtype=torch.float32)
    mp = torch.empty(g.V, device="cuda", dtype=torch.int32)

    def step():
        g.reset_messages()
        g.run_bp(iters, d, T)
        g.get_beliefs(out=q)
        g.decode_map(out=mp)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g.status()

    ms_step = dt * 1e3 / args.steps
    value = spec.num_edge_states * iters * args.steps / dt
    bm = byte_model(spec, iters)
    # live per-launch timing of each phase (HIP events on the library's stream)
    reps = args.phase_reps
    t_var = g.time_phase(0, reps, d, T)
    t_fac = g.time_phase(1, reps, d, T)
    t_it = g.time_phase(2, reps, d, T)
    t_fused = g.time_phase(3, reps, d, T) if g.fused else None
    fl = [l for l in g.launches() if l["phase"] == 1]
    if g.fused and g.fused_in_use:
        # the fused iteration is the dominant (and only) kernel of a solve;
        # it moves the floor bytes: phi, messages in and out, evidence
        kernel, kbytes, kms = "fused iteration (dense pairwise factors, beliefs recomputed)", \
            bm["floor_bytes"], t_fused
        tkey, shape = "fused", (fl[0]["fused_wpb"], fl[0]["fused_variant"])
    elif t_fac >= t_var:
        kernel, kbytes, kms = "factor phase (every factor launch of one iteration)", bm["factor_bytes"], t_fac
        tkey, shape = "factor", (fl[0]["wpb"], fl[0]["swizzle"]) if len(fl) == 1 else (None, None)
    else:
        vl = [l for l in g.launches() if l["phase"] == 0]
        kernel, kbytes, kms = "variable phase (belief sums)", bm["variable_bytes"], t_var
        tkey, shape = "variable", (vl[0]["wpb"], vl[0]["swizzle"]) if len(vl) == 1 else (None, None)
    achieved = kbytes / (kms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, tkey, shape)
    copy_gbps = plain_copy_gbps()
    probes = stream_probes(ctx)
    out = {
        "metric": "edge-state message updates/sec",
        "value": value,
        "unit": "edge-state updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "V": spec.num_vars, "F": spec.num_factors,
                   "edge_states": spec.num_edge_states, "iters": iters, "damping": d,
                   "temperature": T},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                     "algorithmic_bytes_per_launch": kbytes, "avg_launch_ms": kms,
                     "plain_copy_gbps": copy_gbps,
                     "frac_of_plain_copy": achieved / copy_gbps if copy_gbps else None,
                     "frac_of_in_house_mix": achieved / probes["mix5r1w_gbps"],
                     "working_set_bytes": bm["floor_bytes"],
                     "cache_resident": bm["floor_bytes"] < LLC_BYTES,
                     "note": ("the working set fits the 256 MB last-level cache, so this fraction is not an HBM "
                              "claim; roofline_beyond_cache holds the HBM-bound case")
                     if bm["floor_bytes"] < LLC_BYTES else "working set exceeds the last-level cache"},
        "in_house_stream": probes,
        "phases_ms": {"variable": t_var, "factor": t_fac, "two_phase_iteration": t_it, "fused_iteration": t_fused},
        "iteration_gbps": bm["iter_bytes"] / (t_it * 1e-3) / 1e9,
        "solve_gbps": bm["iter_bytes"] * iters / (ms_step * 1e-3) / 1e9,
        "kernel_src_sha": kernel_source_sha(),
        "launch_shapes": [{k: l[k] for k in ("phase", "kind", "a", "b", "wpb", "swizzle", "fused_wpb",
                                              "fused_variant")} for l in g.launches()],
        "tune_source": tuned["source"] if tuned else "default",
        "fused_iterations": g.fused_in_use,
        "device": tune.device_key(0),
    }
    if args.serving:
        out["serving"] = serving_leg(lbp, W, ctx, args.serving,
                                     [int(x) for x in str(args.serving_budget_mb).split(",") if x],
                                     steps=args.serving_steps, slots=args.serving_slots)
    if not args.no_scaleup and args.workload != "potts2048":
        sc = scaleup_leg(lbp, W, ctx, tune)
        out["roofline_beyond_cache"] = sc.pop("roofline")
        out["roofline_beyond_cache"]["frac_of_in_house_mix"] = (out["roofline_beyond_cache"]["achieved"] /
                                                                probes["mix5r1w_gbps"])
        out["potts2048"] = sc
        print("potts2048: %.2f ms per solve, fused launch %.1f us, frac %.3f" % (
            sc["ms_per_solve"], 1e3 * out["roofline_beyond_cache"]["avg_launch_ms"],
            out["roofline_beyond_cache"]["frac"]), file=sys.stderr, flush=True)
    if not args.no_small and args.workload not in ("rbm", "rbm_t005", "deconv"):
        out["small_graphs"] = small_graphs_leg(lbp, W, ctx, tune)
        print("small graphs: RBM %.2f us, deconvolution %.2f us per iteration" % (
            out["small_graphs"]["rbm"]["us_per_iteration"], out["small_graphs"]["deconv"]["us_per_iteration"]),
            file=sys.stderr, flush=True)
    if not args.no_gradient:
        out["gradient"] = gradient_leg(lbp, W, ctx)
    if args.samples:
        out["sampling"] = sampling_leg(lbp, W, ctx, args.samples)
    if args.batch:
        out["batch"] = batch_leg(lbp, W, ctx, args.batch)
    if args.paper_rbm:
        out["paper_rbm"] = paper_rbm_leg(lbp, W, ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, iters, d, T)
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out))
    g.free()
    ctx.close()


if __name__ == "__main__":
    main()
