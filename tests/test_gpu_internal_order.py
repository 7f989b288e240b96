"""Internal variable order on the GPU.  Wide logical factors whose parents are
scattered low-degree variables make the library lay variables out in its own
order; everything that crosses the boundary stays in the caller's order.

The check: the same graph with its variables relabelled by a random
permutation gives bitwise the same results, mapped through the permutation
(beliefs, MAP, messages, results after new evidence, perturb-and-MAP samples,
batched and served results).  Relabelling keeps every variable's edges in the same
order and no variable here has enough edges for column groups, so each
variable's sum runs in the same order in both layouts.  The graph is also
checked against the FP64 oracle over its first iterations."""
import numpy as np
import pytest

from oracle import OracleGraph
from paper_2202_04110_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbp(gpu_lib):
    return gpu_lib


@pytest.fixture(scope="module")
def ctx(lbp):
    return lbp.Context(0)


def scattered_graph(seed, n_par=240, n_wide=8, n_free=70):
    """Binary parents (each in one wide OR/AND and one pairwise factor with a
    free variable of 2-4 states), one binary child per wide factor, and
    pairwise factors among the free variables."""
    rng = np.random.default_rng(seed)
    n_child = n_wide
    ns = np.concatenate([np.full(n_par + n_child, 2), rng.integers(2, 5, n_free)]).astype(np.int32)
    # interleave the three groups so that parents are scattered over the ids
    ids = rng.permutation(len(ns))
    ns = ns[np.argsort(ids)]
    par = ids[:n_par]
    child = ids[n_par:n_par + n_child]
    free = ids[n_par + n_child:]
    ev = rng.normal(0.0, 1.0, int(ns.sum())).astype(np.float32)
    factors = []
    order = rng.permutation(n_par)
    cuts = np.sort(rng.choice(np.arange(12, n_par - 12), n_wide - 1, replace=False))
    for i, grp in enumerate(np.split(order, cuts)):
        factors.append({"kind": W.OR if i % 2 == 0 else W.AND, "vars": list(par[grp]) + [int(child[i])]})
    for p in par:
        f = int(free[rng.integers(0, n_free)])
        factors.append({"kind": W.ENUM, "vars": [int(p), f],
                        "logpot": rng.normal(0.0, 0.8, 2 * int(ns[f])).astype(np.float32)})
    for _ in range(90):
        a, b = rng.choice(free, 2, replace=False)
        factors.append({"kind": W.ENUM, "vars": [int(a), int(b)],
                        "logpot": rng.normal(0.0, 0.8, int(ns[a]) * int(ns[b])).astype(np.float32)})
    return W._general_graph(ns, ev, factors, "scattered wide logical factors")


def wide_parents(spec):
    """Parents of the logical factors with more than 8 edges, in factor order."""
    out = []
    for f in range(spec.num_factors):
        e0, e1 = spec.factor_edge_off[f], spec.factor_edge_off[f + 1]
        if spec.factor_kind[f] != W.ENUM and e1 - e0 > 8:
            out.extend(int(v) for v in spec.edge_var[e0:e1 - 1])
    return out


def relabel(spec, perm):
    """Variable v of spec becomes variable perm[v]; factors keep their order."""
    V = spec.num_vars
    inv = np.argsort(perm)
    ns = spec.var_num_states[inv]
    off = spec.var_state_off()
    ev = np.concatenate([spec.evidence[off[inv[i]]:off[inv[i] + 1]] for i in range(V)])
    out = spec.copy()
    out.var_num_states = np.ascontiguousarray(ns, np.int32)
    out.evidence = np.ascontiguousarray(ev, np.float32)
    out.edge_var = np.ascontiguousarray(perm[spec.edge_var], np.int32)
    return out


def flat_perm(spec, perm):
    """Index array mapping spec's flat variable-state order to the relabelled one."""
    off = spec.var_state_off()
    inv = np.argsort(perm)
    n2 = spec.var_num_states[inv]
    off2 = np.concatenate([[0], np.cumsum(n2)])
    idx = np.empty(spec.num_var_states, np.int64)
    for v in range(spec.num_vars):
        idx[off[v]:off[v + 1]] = off2[perm[v]] + np.arange(off[v + 1] - off[v])
    return idx


@pytest.mark.parametrize("T", [1.0, 0.0])
def test_relabelled_graph_gives_the_same_results(lbp, ctx, T):
    import torch
    spec = scattered_graph(31)
    perm = np.random.default_rng(32).permutation(spec.num_vars)
    spec2 = relabel(spec, perm)
    fidx = flat_perm(spec, perm)
    # both graphs' wide-factor parents are out of order, so both get renumbered
    for sp in (spec, spec2):
        wp = wide_parents(sp)
        assert wp != sorted(wp)
    g, g2 = lbp.Graph(ctx, spec), lbp.Graph(ctx, spec2)
    try:
        for it in (3, 27):
            g.run_bp(it, 0.5, T)
            g2.run_bp(it, 0.5, T)
            q, q2 = g.get_beliefs(), g2.get_beliefs()
            np.testing.assert_array_equal(q, q2[fidx])
            np.testing.assert_array_equal(g.decode_map(), g2.decode_map()[perm])
            np.testing.assert_array_equal(g.get_messages(), g2.get_messages())
        # new evidence, in each graph's own flat order
        ev = np.random.default_rng(33).normal(0.0, 1.5, spec.num_var_states).astype(np.float32)
        ev2 = np.empty_like(ev)
        ev2[fidx] = ev
        g.set_evidence(ev)
        g2.set_evidence(ev2)
        g.run_bp(5, 0.5, T)
        g2.run_bp(5, 0.5, T)
        np.testing.assert_array_equal(g.get_beliefs(), g2.get_beliefs()[fidx])
        np.testing.assert_array_equal(g.decode_map(), g2.decode_map()[perm])
        # perturb-and-MAP: the same noise, each in its graph's flat order
        S = 3
        nz = np.random.default_rng(34).gumbel(size=(S, spec.num_var_states)).astype(np.float32)
        nz2 = np.empty_like(nz)
        nz2[:, fidx] = nz
        s1, s2 = lbp.Sampler(g, S), lbp.Sampler(g2, S)
        m1 = s1.run(20, 0.5, 0.0, torch.from_numpy(nz).cuda()).cpu().numpy()
        m2 = s2.run(20, 0.5, 0.0, torch.from_numpy(nz2).cuda()).cpu().numpy()
        s1.free()
        s2.free()
        np.testing.assert_array_equal(m1, m2[:, perm])
    finally:
        g.free()
        g2.free()


def test_batched_with_a_relabelled_copy(lbp, ctx):
    """A batch holding the graph, its relabelled copy and a Potts grid (in
    the caller's order) gives each graph its lone results."""
    spec = scattered_graph(38)
    perm = np.random.default_rng(39).permutation(spec.num_vars)
    spec2 = relabel(spec, perm)
    fidx = flat_perm(spec, perm)
    grid = W.potts_grid(20, 3, 40)
    lone = []
    for sp in (spec, spec2, grid):
        g = lbp.Graph(ctx, sp)
        g.run_bp(25, 0.5, 0.0)
        lone.append((g.get_beliefs(), g.decode_map()))
        g.free()
    gs = [lbp.Graph(ctx, sp) for sp in (spec, spec2, grid)]
    b = lbp.Batch(ctx, gs)
    try:
        b.run_bp(25, 0.5, 0.0)
        for g, (q, mp) in zip(gs, lone):
            np.testing.assert_array_equal(g.get_beliefs(), q)
            np.testing.assert_array_equal(g.decode_map(), mp)
        np.testing.assert_array_equal(gs[0].get_beliefs(), gs[1].get_beliefs()[fidx])
        np.testing.assert_array_equal(gs[0].decode_map(), gs[1].decode_map()[perm])
    finally:
        b.free()
        for g in gs:
            g.free()


def test_internal_order_against_the_oracle(lbp, ctx):
    """Beliefs and MAP after 1, 2 and 4 sum-product iterations from zero
    messages, against the FP64 oracle in the caller's order."""
    spec = scattered_graph(35)
    og = OracleGraph(spec)
    g = lbp.Graph(ctx, spec)
    try:
        for it in (1, 2, 4):
            g.reset_messages()
            g.run_bp(it, 0.5, 1.0)
            _, qo, mo = og.beliefs(og.run(it, 0.5, 1.0), 1.0)
            q = g.get_beliefs()
            assert np.abs(q - qo).max() < 1e-4, (it, np.abs(q - qo).max())
            # MAP where the oracle's margin is clear
            off = spec.var_state_off()
            mp = g.decode_map()
            for v in range(spec.num_vars):
                row = np.sort(qo[off[v]:off[v + 1]])
                if row[-1] - row[-2] > 1e-3:
                    assert mp[v] == mo[v], (it, v)
    finally:
        g.free()


def test_served_results_in_the_callers_order(lbp, ctx):
    """Served requests (their evidence and tables scattered into panels on
    the device) match lone runs of the same graph and of its relabelling."""
    from paper_2202_04110_amd.serving import run_stream
    spec = scattered_graph(36)
    perm = np.random.default_rng(37).permutation(spec.num_vars)
    spec2 = relabel(spec, perm)
    fidx = flat_perm(spec, perm)
    srv = lbp.Server(ctx, budget_bytes=64 << 20, max_slots=4, steps_per_round=5)
    res, summ = run_stream(srv, [spec, spec2], np.zeros(2), 30, 0.5, 1.0, timeout=120)
    srv.close()
    assert summ["ok"] == 2
    g = lbp.Graph(ctx, spec)
    g.run_bp(30, 0.5, 1.0)
    q, mp = g.get_beliefs(), g.decode_map()
    g.free()
    np.testing.assert_array_equal(res[0]["beliefs"], q)
    np.testing.assert_array_equal(res[0]["map"], mp)
    np.testing.assert_array_equal(res[1]["beliefs"][fidx], q)
    np.testing.assert_array_equal(res[1]["map"][perm], mp)
