"""Stored expected values (tests/golden/*.json, written by
tests/golden/make_golden.py with the FP64 oracle only).

Pins of the stored values against the mathematics, not against the oracle:
on the tree-structured cases BP is exact, so the stored normalised beliefs
must equal brute-force T-marginals (max-marginal offsets at T = 0) and the
stored MAP the brute-force MAP; on the loopy cases the stored run must have
converged (final residual below 1e-9), so the stored beliefs are those of a
fixed point.  The oracle must reproduce every file (a change to its
arithmetic shows here first), and the HIP path is compared with the stored
values directly (q within 1e-4, MAP equal)."""
import glob
import json
import os

import numpy as np
import pytest

import brute
from paper_2202_04110_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
FILES = sorted(glob.glob(os.path.join(HERE, "golden", "*.json")))
NAMES = [os.path.splitext(os.path.basename(f))[0] for f in FILES]


def _load(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as fh:
        doc = json.load(fh)
    g = W.GraphSpec(**{k: np.asarray(v) for k, v in doc["graph"].items()}, name=name)
    return doc, g


def test_golden_files_present():
    assert len(NAMES) >= 8
    for n in NAMES:
        doc, _ = _load(n)
        assert doc["citation"].startswith("Sec. ")


@pytest.mark.parametrize("name", NAMES)
def test_stored_values_pinned(name):
    doc, g = _load(name)
    q = np.asarray(doc["q"])
    T = doc["temperature"]
    if doc["tree"]:
        np.testing.assert_allclose(q, brute.exact_q(g, T), rtol=0, atol=1e-9)
        if T == 0.0:
            x, _ = brute.exact_map(g)
            np.testing.assert_array_equal(np.asarray(doc["map"]), x)
    else:
        assert doc["final_residual"] < 1e-9
    # every row of q is a normalised log-distribution (T > 0) or has max 0
    off = g.var_state_off()
    for v in range(g.num_vars):
        row = q[off[v]:off[v + 1]]
        if T > 0:
            assert abs(T * np.log(np.sum(np.exp(row / T)))) < 1e-9
        else:
            assert abs(row.max()) < 1e-12
        assert doc["map"][v] == int(np.argmax(row))
        top = np.sort(row)
        assert top[-1] - top[-2] > 1e-3  # no near-tie: MAP comparisons are well posed


@pytest.mark.parametrize("name", NAMES)
def test_oracle_reproduces_stored_values(name):
    from oracle import OracleGraph
    doc, g = _load(name)
    og = OracleGraph(g)
    m = og.run(doc["iters"], doc["damping"], doc["temperature"])
    _, q, mp = og.beliefs(m, doc["temperature"])
    np.testing.assert_allclose(q, np.asarray(doc["q"]), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(mp, np.asarray(doc["map"]))


@pytest.mark.gpu
@pytest.mark.parametrize("name", NAMES)
def test_hip_path_matches_stored_values(gpu_lib, name):
    lbp = gpu_lib
    doc, g = _load(name)
    ctx = lbp.Context(0)
    gr = lbp.Graph(ctx, g)
    gr.run_bp(doc["iters"], doc["damping"], doc["temperature"])
    q = gr.get_beliefs()
    np.testing.assert_allclose(q, np.asarray(doc["q"]), rtol=0, atol=1e-4)
    np.testing.assert_array_equal(gr.decode_map(), np.asarray(doc["map"]))
    gr.free()
    ctx.close()
