"""Scheduler of the serving loop on the host (bookkeeping-only executor, no
GPU): admission under the memory budget and slot limit, first-in first-out
queueing, rejection of requests larger than the budget, cancellation, and
malformed requests."""
import time

import numpy as np
import pytest

from paper_2202_04110_amd import workloads as W


@pytest.fixture(scope="module")
def lbp():
    from paper_2202_04110_amd import lbp as mod
    return mod


def _sizes(lbp, spec):
    return lbp.check_layout(spec)


def test_budget_and_slots_respected(lbp):
    specs = [W.potts_grid(L, n, seed=i) for i, (L, n) in enumerate(
        [(20, 3), (40, 5), (12, 8), (60, 2), (30, 4), (25, 6), (50, 3), (16, 2)] * 3)]
    budget = 6 << 20
    srv = lbp.Server(budget_bytes=budget, max_slots=3, steps_per_round=4, host_only=True)
    for i, s in enumerate(specs):
        srv.submit(s, 20, 0.5, 1.0, req_id=i)
    srv.drain(30)
    recs = {r["req_id"]: r for r in srv.poll(1000)}
    st = srv.stats()
    srv.close()
    assert len(recs) == len(specs) and all(r["status"] == 0 for r in recs.values())
    assert st["max_resident"] <= 3
    assert 0 < st["arena_peak_bytes"] <= budget
    assert st["completed"] == len(specs) and st["rounds"] > 0
    # first in, first out: admission times follow submission order
    adm = [recs[i]["t_admit"] for i in range(len(specs))]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    # each request was prepared after it arrived and admitted after that
    for r in recs.values():
        assert r["t_arrival"] <= r["t_ready"] <= r["t_admit"] <= r["t_done"]
    assert st["prep_threads"] >= 1 and st["prep_us"] > 0 and st["round_us"] <= st["busy_us"]
    assert st["launch_us"] <= st["round_us"] and st["finish_us"] <= st["busy_us"] and st["admit_us"] > 0
    # zero-filled outputs of the right sizes from the bookkeeping executor
    assert recs[3]["beliefs"].shape == (specs[3].num_var_states,)
    assert recs[3]["map"].shape == (specs[3].num_vars,)


def test_oversized_request_rejected(lbp):
    srv = lbp.Server(budget_bytes=1 << 20, max_slots=4, host_only=True)
    srv.submit(W.potts_grid(200, 8, seed=1), 10, 0.5, 1.0, req_id=1)
    srv.submit(W.potts_grid(10, 3, seed=2), 10, 0.5, 1.0, req_id=2)
    srv.drain(10)
    recs = {r["req_id"]: r for r in srv.poll()}
    assert recs[1]["status"] == lbp.LBP_E_BUDGET and recs[1]["beliefs"] is None
    assert recs[2]["status"] == 0
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 1 and st["failed"] == 0
    srv.close()


def test_malformed_and_invalid_requests(lbp):
    srv = lbp.Server(budget_bytes=1 << 24, host_only=True)
    bad = W.potts_grid(5, 3, seed=1)
    bad.edge_var[0] = 10 ** 6  # caught by the prep threads' validation
    srv.submit(bad, 10, 0.5, 1.0, req_id=7)
    srv.drain(10)
    rec = srv.poll()
    assert rec[0]["req_id"] == 7 and rec[0]["status"] == lbp.LBP_E_INVALID and rec[0]["beliefs"] is None
    assert srv.stats()["failed"] == 1
    bad2 = W.potts_grid(5, 3, seed=1)
    bad2.var_num_states[0] = 1  # caught at submit
    with pytest.raises(lbp.LBPError) as ei:
        srv.submit(bad2, 10, 0.5, 1.0)
    assert ei.value.code == lbp.LBP_E_INVALID
    with pytest.raises(lbp.LBPError) as ei:
        srv.submit(W.potts_grid(5, 3, seed=1), 10, 1.5, 1.0)
    assert ei.value.code == lbp.LBP_E_INVALID
    # backward needs T > 0 and enumeration factors only
    g = W.potts_grid(5, 3, seed=1)
    with pytest.raises(lbp.LBPError) as ei:
        srv.submit(g, 10, 0.5, 0.0, grad_q=np.zeros(g.num_var_states))
    assert ei.value.code == lbp.LBP_E_INVALID
    lg = W.single_logical(1, W.OR, 3)
    with pytest.raises(lbp.LBPError) as ei:
        srv.submit(lg, 10, 0.5, 1.0, grad_q=np.zeros(lg.num_var_states))
    assert ei.value.code == lbp.LBP_E_UNSUPPORTED
    assert srv.stats()["accepted"] == 1
    srv.close()


def test_queue_waits_for_memory_then_admits(lbp):
    """A budget that holds one graph at a time: requests wait in the queue and
    are admitted one by one as memory frees up."""
    spec = W.potts_grid(40, 5, seed=3)
    srv0 = lbp.Server(budget_bytes=1 << 30, host_only=True)
    srv0.submit(spec, 1, 0.5, 1.0, req_id=0)
    srv0.drain(10)
    one = srv0.stats()["arena_peak_bytes"]  # bytes of one request
    srv0.close()
    assert one > 0
    srv = lbp.Server(budget_bytes=int(one * 1.5), max_slots=8, steps_per_round=3, host_only=True)
    for i in range(5):
        srv.submit(spec, 9, 0.5, 1.0, req_id=i)
    srv.drain(10)
    recs = {r["req_id"]: r for r in srv.poll()}
    st = srv.stats()
    srv.close()
    assert st["max_resident"] == 1 and st["completed"] == 5
    # each request is admitted only after the previous one finished
    for i in range(4):
        assert recs[i + 1]["t_admit"] >= recs[i]["t_done"]


def test_cancel_queued_request(lbp):
    spec = W.potts_grid(30, 4, seed=4)
    srv = lbp.Server(budget_bytes=1 << 30, max_slots=1, steps_per_round=1, host_only=True)
    for i in range(4):
        srv.submit(spec, 5000, 0.5, 1.0, req_id=i)
    srv.cancel(3)
    srv.cancel(0)
    srv.drain(60)
    recs = {r["req_id"]: r for r in srv.poll()}
    st = srv.stats()
    srv.close()
    assert recs[3]["status"] == lbp.LBP_E_STATE and recs[3]["beliefs"] is None
    assert recs[0]["status"] in (0, lbp.LBP_E_STATE)
    assert recs[1]["status"] == 0 and recs[2]["status"] == 0
    assert st["cancelled"] >= 1


def test_stream_driver_host_only(lbp):
    from paper_2202_04110_amd.serving import run_stream
    reqs = W.served_requests(24, seed=5, max_side=48)
    specs = [W.request_graph(r) for r in reqs]
    arr = W.poisson_arrivals(len(reqs), qps=400.0, seed=5)
    srv = lbp.Server(budget_bytes=64 << 20, max_slots=8, steps_per_round=5, host_only=True)
    res, summ = run_stream(srv, specs, arr, 50, 0.5, 1.0, timeout=30)
    srv.close()
    assert summ["ok"] == 24 and summ["p99_s"] >= summ["p50_s"] >= 0


def test_early_exit_requests_host_only(lbp):
    """Requests with a tolerance (lbp_server_submit_until) on the bookkeeping
    executor, whose messages stay zero and so measure a residual of 0 at
    every check: with tol > 0 they leave at their first check point (after
    check_every iterations, or max_iters if fewer), with tol = 0 (0 < 0 is
    false) they run to max_iters; plain requests report every iteration and
    residual -1.  Rounds stop at each request's own check points, so
    iters_done is exactly the check point, not a multiple of the round."""
    srv = lbp.Server(budget_bytes=64 << 20, max_slots=8, steps_per_round=4, host_only=True)
    spec = W.potts_grid(12, 3, seed=1)
    cases = {1: (50, 1e-3, 7), 2: (5, 1e-3, 7), 3: (30, 0.0, 7), 4: (26, 1e-3, 1), 5: (40, None, 10)}
    for rid, (iters, tol, ce) in cases.items():
        srv.submit(spec, iters, 0.5, 1.0, req_id=rid, tol=tol, check_every=ce)
    srv.drain(30)
    recs = {r["req_id"]: r for r in srv.poll()}
    srv.close()
    assert all(r["status"] == 0 for r in recs.values())
    assert recs[1]["iters"] == 7 and recs[1]["residual"] == 0.0
    assert recs[2]["iters"] == 5
    assert recs[3]["iters"] == 30 and recs[3]["residual"] == 0.0
    assert recs[4]["iters"] == 1
    assert recs[5]["iters"] == 40 and recs[5]["residual"] == -1.0


def test_early_exit_argument_errors(lbp):
    srv = lbp.Server(budget_bytes=8 << 20, max_slots=2, host_only=True)
    spec = W.potts_grid(8, 2, seed=3)
    for tol, ce in ((-1.0, 5), (float("nan"), 5), (float("inf"), 5), (1e-3, 0)):
        with pytest.raises(lbp.LBPError) as ei:
            srv.submit(spec, 10, 0.5, 1.0, tol=tol, check_every=ce)
        assert ei.value.code == lbp.LBP_E_INVALID
    with pytest.raises(ValueError):
        srv.submit(spec, 10, 0.5, 1.0, grad_q=np.zeros(spec.num_var_states, np.float32), tol=1e-3)
    assert srv.stats()["accepted"] == 0
    srv.close()
