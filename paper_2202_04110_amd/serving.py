"""Serving driver: submits requests at scheduled arrival times and reports
latency percentiles and throughput.  The scheduling itself (admission by
memory budget, resident messages, shared multi-graph launches) is the
library's worker thread; this module only plays the clients."""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def run_stream(server, specs, arrivals, iters: int, damping: float, temperature: float, grad_qs=None,
               ckpt_every: int = 10, timeout: float = 900.0, start_delay: float = 0.05, clients: int = 4,
               tol=None, check_every: int = 5):
    """Submits request i (graph specs[i]) at server-clock time
    start + arrivals[i] seconds, with its latency measured from that scheduled
    time; ``clients`` threads perform the submissions (each copies its
    request's arrays into the server).  grad_qs[i] (or None) asks for the
    log-potential gradient.  tol (not None): requests without a gradient stop
    once their residual, checked every check_every iterations, is below tol
    (at most ``iters``).  Returns (results by request id, summary)."""
    n = len(specs)
    order = np.argsort(arrivals, kind="stable")
    t_start = server.clock() + start_delay
    results = {}

    def collect():
        for rec in server.poll(256):
            results[rec["req_id"]] = rec

    pool = ThreadPoolExecutor(max_workers=max(1, clients))
    futures = []
    for i in order:
        due = t_start + float(arrivals[i])
        while True:
            now = server.clock()
            if now >= due:
                break
            collect()
            time.sleep(min(0.002, due - now))
        gq = None if grad_qs is None else grad_qs[i]
        t = tol if gq is None else None
        futures.append(pool.submit(server.submit, specs[i], iters, damping, temperature, gq, ckpt_every, due,
                                   int(i), t, check_every))
    for f in futures:
        f.result()
    pool.shutdown()
    server.drain(timeout)
    collect()
    while len(results) < n:
        got = server.poll(256)
        if not got:
            break
        for rec in got:
            results[rec["req_id"]] = rec
    ok = [r for r in results.values() if r["status"] == 0]
    lat = np.array([r["t_done"] - r["t_arrival"] for r in ok]) if ok else np.zeros(0)
    makespan = (max(r["t_done"] for r in ok) - t_start) if ok else 0.0
    es_total = sum(int(specs[r["req_id"]].num_edge_states) * r["iters"] for r in ok)
    def p50(xs):
        return float(np.percentile(np.array(xs), 50)) if xs else None

    summary = {
        "requests": n, "ok": len(ok),
        "iters_mean": float(np.mean([r["iters"] for r in ok])) if ok else None,
        "prep_p50_s": p50([r["t_ready"] - r["t_arrival"] for r in ok]),
        "admit_wait_p50_s": p50([r["t_admit"] - r["t_ready"] for r in ok]),
        "service_p50_s": p50([r["t_done"] - r["t_admit"] for r in ok]),
        "last_ready_s": (max(r["t_ready"] for r in ok) - t_start) if ok else None,
        "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_s": float(lat.mean()) if lat.size else None,
        "makespan_s": makespan,
        "requests_per_s": len(ok) / makespan if makespan > 0 else None,
        "edge_state_updates_per_s": es_total / makespan if makespan > 0 else None,
        "stats": server.stats(),
    }
    return results, summary
