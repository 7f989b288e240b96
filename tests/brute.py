"""Brute-force enumeration over all joint states of a tiny factor graph.

Independent of both the oracle and the HIP path: it never passes messages, it
evaluates the joint log-score of every assignment and marginalises directly.
On a tree, loopy BP is exact (textbook result for BP on tree-structured factor
graphs), so its fixed point must reproduce these numbers.
"""
from __future__ import annotations

import numpy as np

ENUM, OR, AND = 0, 1, 2


def _factor_configs(g, f):
    """(states array (C, k), log-potentials (C,)) of enumeration factor f."""
    e0, e1 = g.factor_edge_off[f], g.factor_edge_off[f + 1]
    vs = g.edge_var[e0:e1]
    ns = [int(g.var_num_states[v]) for v in vs]
    t = g.factor_cfg_table[f]
    lp = g.log_potentials[g.logpot_off[f]:g.logpot_off[f + 1]].astype(np.float64)
    if g.cfg_table_num_cfgs[t] == 0:
        cfg = np.array(np.unravel_index(np.arange(int(np.prod(ns))), ns)).T
    else:
        k = g.cfg_table_arity[t]
        cfg = g.cfg_table_states[g.cfg_table_off[t]:g.cfg_table_off[t + 1]].reshape(-1, k)
    return vs, cfg, lp


def joint_scores(g):
    """All assignments X (N, V) and their log-scores (N,), -inf when invalid."""
    ns = [int(n) for n in g.var_num_states]
    N = int(np.prod(ns))
    X = np.array(np.unravel_index(np.arange(N), ns)).T.astype(np.int64)
    vs_off = np.concatenate([[0], np.cumsum(ns)])
    ev = g.evidence.astype(np.float64)
    sc = np.zeros(N)
    for v in range(len(ns)):
        sc += ev[vs_off[v] + X[:, v]]
    for f in range(g.factor_kind.shape[0]):
        e0, e1 = g.factor_edge_off[f], g.factor_edge_off[f + 1]
        vs = g.edge_var[e0:e1]
        if g.factor_kind[f] == ENUM:
            _, cfg, lp = _factor_configs(g, f)
            lookup = {tuple(int(x) for x in c): lp[i] for i, c in enumerate(cfg)}
            sub = X[:, vs]
            sc += np.array([lookup.get(tuple(r), -np.inf) for r in sub])
        else:
            par = X[:, vs[:-1]] != 0
            child = X[:, vs[-1]] != 0
            val = par.any(1) if g.factor_kind[f] == OR else par.all(1)
            sc = np.where(val == child, sc, -np.inf)
    return X, sc


def _lse(x, T, axis=None):
    x = np.asarray(x, np.float64)
    if T == 0:
        return np.max(x, axis=axis)
    M = np.max(x, axis=axis, keepdims=True)
    Ms = np.where(np.isfinite(M), M, 0.0)
    r = Ms + T * np.log(np.sum(np.exp((x - Ms) / T), axis=axis, keepdims=True))
    return np.squeeze(r, axis=axis) if axis is not None else float(r.reshape(()))


def exact_q(g, T):
    """q[v,s] = LSE_T{score(x): x_v = s} - LSE_T{score(x)}: T-scaled log
    marginals (T > 0) or max-marginal offsets (T = 0), variable-major."""
    X, sc = joint_scores(g)
    Z = _lse(sc, T)
    out = []
    for v in range(g.var_num_states.shape[0]):
        for s in range(int(g.var_num_states[v])):
            out.append(_lse(sc[X[:, v] == s], T) - Z)
    return np.asarray(out)


def exact_map(g):
    X, sc = joint_scores(g)
    i = int(np.argmax(sc))
    return X[i].astype(np.int32), float(sc[i])


def marginal_probs(g, T):
    """p_T(x) for every assignment."""
    X, sc = joint_scores(g)
    w = np.exp((sc - sc.max()) / T)
    return X, w / w.sum()


def factor_update(g, f, n_rows, T):
    """u[e_j, s] of factor f for incoming rows n_rows (list of arrays, one per
    edge of f), by enumerating the factor's valid joint states: LSE_T over the
    joint states with slot j in state s of (potential + incoming of the other
    slots).  Returns a list of arrays, each shifted so that its max is 0."""
    e0, e1 = g.factor_edge_off[f], g.factor_edge_off[f + 1]
    vs = g.edge_var[e0:e1]
    k = len(vs)
    ns = [int(g.var_num_states[v]) for v in vs]
    if g.factor_kind[f] == ENUM:
        _, cfg, lp = _factor_configs(g, f)
    else:
        full = np.array(np.unravel_index(np.arange(int(np.prod(ns))), ns)).T
        par = full[:, :-1] != 0
        val = par.any(1) if g.factor_kind[f] == OR else par.all(1)
        cfg = full[val == (full[:, -1] != 0)]
        lp = np.zeros(cfg.shape[0])
    out = []
    for j in range(k):
        u = np.empty(ns[j])
        for s in range(ns[j]):
            rows = cfg[:, j] == s
            tot = lp[rows].copy()
            for l in range(k):
                if l != j:
                    tot += n_rows[l][cfg[rows, l]]
            u[s] = _lse(tot, T)
        out.append(u - u.max())
    return out


def rbm_exact_map(nv, nh, w, bv, bh):
    """Exact MAP of a binary RBM with score sum bv x + sum bh h + x^T W h:
    enumerate the visible states and set each hidden unit optimally."""
    best, arg = -np.inf, None
    chunk = 4096
    for start in range(0, 1 << nv, chunk):
        idx = np.arange(start, min(start + chunk, 1 << nv))
        Xv = ((idx[:, None] >> np.arange(nv - 1, -1, -1)) & 1).astype(np.float64)
        act = Xv @ w + bh[None, :]
        sc = Xv @ bv + np.maximum(act, 0).sum(1)
        i = int(np.argmax(sc))
        if sc[i] > best:
            best = float(sc[i])
            arg = np.concatenate([Xv[i], (act[i] > 0).astype(np.float64)]).astype(np.int32)
    return arg, best
