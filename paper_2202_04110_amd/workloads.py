"""Seeded synthetic factor graphs in the flat-array form the C-ABI uploads.

This module holds input generation only: it draws random numbers and lays out
index arrays.  It performs none of the message-passing arithmetic, so both the
HIP path and the FP64 oracle can take their inputs from it.

Array form (mirrors ``lbp_graph_desc`` in ``include/lbp.h``):

* ``var_num_states[V]``  int32, every entry >= 2 (variables with a varying
  number of states, Sec. "Package features").
* ``evidence[VS]``       float32, unary log-potentials, variable-major:
  the states of variable v sit at ``sum(var_num_states[:v]) + s``.
* ``factor_kind[F]``     int32, 0 = enumeration factor, 1 = OR, 2 = AND.
* ``factor_edge_off[F+1]`` int64, the edges of factor f are
  ``factor_edge_off[f] .. factor_edge_off[f+1]-1``.
* ``edge_var[E]``        int32, variable of each edge.  For OR/AND factors the
  last edge of the factor is the child, the others are the parents.
* ``factor_cfg_table[F]`` int32, configuration table of an enumeration factor
  (-1 for logical factors).
* ``cfg_table_num_cfgs[NT]`` int32, 0 marks a dense table: every joint state of
  the factor's variables, row-major (last variable fastest).
* ``cfg_table_arity[NT]`` int32.
* ``cfg_table_off[NT+1]`` int64, offsets into ``cfg_table_states``.
* ``cfg_table_states``   int32, explicit tables: ``num_cfgs x arity`` states.
* ``logpot_off[F+1]``    int64, offsets into ``log_potentials``; an
  enumeration factor holds one log-potential per valid configuration (Sec.
  "Specifying complex factor graphs": factors given by their valid
  configurations), a logical factor holds none.
* ``log_potentials[Tn]`` float32.

Flat message arrays (Sec. "A fully flat array-based LBP implementation") are
indexed edge-major in factor order: edge e owns ``var_num_states[edge_var[e]]``
consecutive entries.

Every workload below follows the recipe stated for it; ``N(mu, s)`` means a
normal draw with standard deviation ``s``.  Draw order: evidence in variable
order, then tables in factor order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ENUM, OR, AND = 0, 1, 2


@dataclass
class GraphSpec:
    var_num_states: np.ndarray
    evidence: np.ndarray
    factor_kind: np.ndarray
    factor_edge_off: np.ndarray
    edge_var: np.ndarray
    factor_cfg_table: np.ndarray
    cfg_table_num_cfgs: np.ndarray
    cfg_table_arity: np.ndarray
    cfg_table_off: np.ndarray
    cfg_table_states: np.ndarray
    logpot_off: np.ndarray
    log_potentials: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.var_num_states = np.ascontiguousarray(self.var_num_states, np.int32)
        self.evidence = np.ascontiguousarray(self.evidence, np.float32)
        self.factor_kind = np.ascontiguousarray(self.factor_kind, np.int32)
        self.factor_edge_off = np.ascontiguousarray(self.factor_edge_off, np.int64)
        self.edge_var = np.ascontiguousarray(self.edge_var, np.int32)
        self.factor_cfg_table = np.ascontiguousarray(self.factor_cfg_table, np.int32)
        self.cfg_table_num_cfgs = np.ascontiguousarray(self.cfg_table_num_cfgs, np.int32)
        self.cfg_table_arity = np.ascontiguousarray(self.cfg_table_arity, np.int32)
        self.cfg_table_off = np.ascontiguousarray(self.cfg_table_off, np.int64)
        self.cfg_table_states = np.ascontiguousarray(self.cfg_table_states, np.int32)
        self.logpot_off = np.ascontiguousarray(self.logpot_off, np.int64)
        self.log_potentials = np.ascontiguousarray(self.log_potentials, np.float32)

    # sizes -----------------------------------------------------------------
    @property
    def num_vars(self) -> int:
        return int(self.var_num_states.shape[0])

    @property
    def num_factors(self) -> int:
        return int(self.factor_kind.shape[0])

    @property
    def num_edges(self) -> int:
        return int(self.edge_var.shape[0])

    @property
    def num_var_states(self) -> int:
        return int(self.var_num_states.sum(dtype=np.int64))

    @property
    def num_edge_states(self) -> int:
        return int(self.var_num_states[self.edge_var].sum(dtype=np.int64))

    @property
    def num_logpots(self) -> int:
        return int(self.log_potentials.shape[0])

    def var_state_off(self) -> np.ndarray:
        off = np.zeros(self.num_vars + 1, np.int64)
        np.cumsum(self.var_num_states, out=off[1:])
        return off

    def edge_state_off(self) -> np.ndarray:
        off = np.zeros(self.num_edges + 1, np.int64)
        np.cumsum(self.var_num_states[self.edge_var], out=off[1:])
        return off

    def copy(self) -> "GraphSpec":
        kw = {k: getattr(self, k).copy() for k in ARRAY_FIELDS}
        return GraphSpec(name=self.name, meta=dict(self.meta), **kw)


ARRAY_FIELDS = (
    "var_num_states", "evidence", "factor_kind", "factor_edge_off", "edge_var",
    "factor_cfg_table", "cfg_table_num_cfgs", "cfg_table_arity", "cfg_table_off",
    "cfg_table_states", "logpot_off", "log_potentials",
)


# ---------------------------------------------------------------------------
# builders
# ---------------------------------------------------------------------------
def _pairwise_graph(nstates, evidence, pairs, tables, name, meta=None):
    """Graph whose factors are all dense pairwise enumeration factors.

    ``pairs`` is (F, 2) variable indices, ``tables`` is (F, n_a*n_b) log-potentials
    in row-major order (state of the first variable slowest)."""
    pairs = np.asarray(pairs, np.int64)
    F = pairs.shape[0]
    tables = np.asarray(tables, np.float32).reshape(F, -1)
    return GraphSpec(
        var_num_states=nstates,
        evidence=evidence,
        factor_kind=np.zeros(F, np.int32),
        factor_edge_off=np.arange(F + 1, dtype=np.int64) * 2,
        edge_var=pairs.reshape(-1),
        factor_cfg_table=np.zeros(F, np.int32),
        cfg_table_num_cfgs=np.zeros(1, np.int32),
        cfg_table_arity=np.full(1, 2, np.int32),
        cfg_table_off=np.zeros(2, np.int64),
        cfg_table_states=np.zeros(0, np.int32),
        logpot_off=np.arange(F + 1, dtype=np.int64) * tables.shape[1],
        log_potentials=tables.reshape(-1),
        name=name,
        meta=meta or {},
    )


def grid_pairs(L: int) -> np.ndarray:
    """4-neighbour grid edges on an L x L lattice, variables row-major.

    All horizontal pairs (r,c)-(r,c+1) come first, then all vertical pairs
    (r,c)-(r+1,c)."""
    idx = np.arange(L * L, dtype=np.int64).reshape(L, L)
    h = np.stack([idx[:, :-1].reshape(-1), idx[:, 1:].reshape(-1)], 1)
    v = np.stack([idx[:-1, :].reshape(-1), idx[1:, :].reshape(-1)], 1)
    return np.concatenate([h, v], 0)


def ising_grid(L: int = 32, seed: int = 1) -> GraphSpec:
    """2-D Ising grid: binary variables, unary log-potentials N(0,1) for both
    states, one coupling J ~ N(0, 0.5) per edge with table [[J,-J],[-J,J]]."""
    rng = np.random.default_rng(seed)
    V = L * L
    ev = rng.normal(0.0, 1.0, size=V * 2).astype(np.float32)
    pairs = grid_pairs(L)
    J = rng.normal(0.0, 0.5, size=pairs.shape[0])
    tab = np.stack([J, -J, -J, J], 1)
    return _pairwise_graph(np.full(V, 2, np.int32), ev, pairs, tab, f"ising{L}",
                           {"L": L, "n": 2, "seed": seed})


def potts_grid(L: int = 512, n: int = 5, seed: int = 2, diag: float = 1.0,
               off_sd: float = 0.2) -> GraphSpec:
    """2-D Potts grid: n states, unary N(0,1), per-factor n x n table with
    ``diag`` on the diagonal and N(0, off_sd) elsewhere."""
    rng = np.random.default_rng(seed)
    V = L * L
    ev = rng.normal(0.0, 1.0, size=V * n).astype(np.float32)
    pairs = grid_pairs(L)
    F = pairs.shape[0]
    tab = rng.normal(0.0, off_sd, size=(F, n, n)).astype(np.float32)
    ii = np.arange(n)
    tab[:, ii, ii] = diag
    return _pairwise_graph(np.full(V, n, np.int32), ev, pairs, tab.reshape(F, n * n),
                           f"potts{L}x{n}", {"L": L, "n": n, "seed": seed})


def random_pairwise(seed: int, num_vars: int, num_factors: int, n: int = 4, max_degree: int = 12,
                    ev_sd: float = 1.0, lp_sd: float = 1.0) -> GraphSpec:
    """Loopy pairwise graph with no spatial locality: each factor joins two
    distinct variables drawn uniformly (redrawn while either already has
    ``max_degree`` edges); n states everywhere, evidence N(0, ev_sd), tables
    N(0, lp_sd)."""
    rng = np.random.default_rng(seed)
    deg = np.zeros(num_vars, np.int64)
    pairs = []
    while len(pairs) < num_factors:
        a, b = rng.integers(0, num_vars, size=2)
        if a == b or deg[a] >= max_degree or deg[b] >= max_degree:
            continue
        deg[a] += 1
        deg[b] += 1
        pairs.append((a, b))
    ev = rng.normal(0.0, ev_sd, size=num_vars * n).astype(np.float32)
    tab = rng.normal(0.0, lp_sd, size=(num_factors, n * n)).astype(np.float32)
    return _pairwise_graph(np.full(num_vars, n, np.int32), ev, np.array(pairs, np.int64), tab,
                           f"randpair{num_vars}x{n}", {"seed": seed})


def triplet_grid(L: int = 256, n: int = 3, seed: int = 12, sd: float = 0.5) -> GraphSpec:
    """Higher-order grid: L x L variables with n states, one dense three-way
    factor per three consecutive variables along every row (r,c),(r,c+1),(r,c+2)
    (all row triples first) and every column; evidence N(0,1), tables N(0, sd)
    (n^3 entries, last slot fastest)."""
    rng = np.random.default_rng(seed)
    V = L * L
    ev = rng.normal(0.0, 1.0, size=V * n).astype(np.float32)
    idx = np.arange(V, dtype=np.int64).reshape(L, L)
    h = np.stack([idx[:, :-2], idx[:, 1:-1], idx[:, 2:]], -1).reshape(-1, 3)
    v = np.stack([idx[:-2, :], idx[1:-1, :], idx[2:, :]], -1).reshape(-1, 3)
    tri = np.concatenate([h, v], 0)
    F = tri.shape[0]
    tab = rng.normal(0.0, sd, size=(F, n ** 3)).astype(np.float32)
    return GraphSpec(
        var_num_states=np.full(V, n, np.int32), evidence=ev,
        factor_kind=np.zeros(F, np.int32),
        factor_edge_off=np.arange(F + 1, dtype=np.int64) * 3,
        edge_var=tri.reshape(-1).astype(np.int32),
        factor_cfg_table=np.zeros(F, np.int32),
        cfg_table_num_cfgs=np.zeros(1, np.int32),
        cfg_table_arity=np.full(1, 3, np.int32),
        cfg_table_off=np.zeros(2, np.int64),
        cfg_table_states=np.zeros(0, np.int32),
        logpot_off=np.arange(F + 1, dtype=np.int64) * n ** 3,
        log_potentials=tab.reshape(-1),
        name=f"triplet{L}x{n}", meta={"L": L, "n": n, "seed": seed},
    )


def rbm(nv: int = 784, nh: int = 500, seed: int = 3, w_sd: float = 0.05,
        b_sd: float = 0.1) -> GraphSpec:
    """Restricted Boltzmann machine as a factor graph: visible 0..nv-1, hidden
    nv..nv+nh-1, every visible-hidden pair one factor (visible-major), table
    [[0,0],[0,w]] with w ~ N(0, w_sd); evidence [0, b] with b ~ N(0, b_sd)."""
    rng = np.random.default_rng(seed)
    V = nv + nh
    b = rng.normal(0.0, b_sd, size=V).astype(np.float32)
    ev = np.zeros((V, 2), np.float32)
    ev[:, 1] = b
    i = np.repeat(np.arange(nv, dtype=np.int64), nh)
    j = np.tile(np.arange(nh, dtype=np.int64), nv) + nv
    pairs = np.stack([i, j], 1)
    w = rng.normal(0.0, w_sd, size=pairs.shape[0]).astype(np.float32)
    tab = np.zeros((pairs.shape[0], 4), np.float32)
    tab[:, 3] = w
    return _pairwise_graph(np.full(V, 2, np.int32), ev.reshape(-1), pairs, tab,
                           f"rbm{nv}x{nh}", {"nv": nv, "nh": nh, "seed": seed})


def deconv(seed: int = 4, K: int = 5, tw: int = 6, sd: int = 29, img: int = 32,
           w_p: float = 0.3, s_p: float = 0.01, lam_mu: float = -2.0,
           lam_sd: float = 0.5, clamp: float = 10.0) -> GraphSpec:
    """2-D blind binary deconvolution with logical factors.

    Latent templates W (K x tw x tw) and activations S (K x sd x sd); for every
    pair (S_k[p,q], W_k[a,b]) that lands inside the img x img image a product
    variable SW = AND(S, W); every pixel X_ij = OR of the SW landing on it.
    Evidence: S and W get [0, lambda], lambda ~ N(lam_mu, lam_sd); SW gets 0;
    X is clamped to the image drawn from ground truth W ~ Bernoulli(w_p),
    S ~ Bernoulli(s_p) with [0, +-clamp].

    Variables: W, S, SW, X.  Factors: all AND (edges S, W, child SW), then all
    OR (parents SW in creation order, child X)."""
    rng = np.random.default_rng(seed)
    nW, nS = K * tw * tw, K * sd * sd
    lam = rng.normal(lam_mu, lam_sd, size=nW + nS).astype(np.float32)
    gtW = (rng.random((K, tw, tw)) < w_p)
    gtS = (rng.random((K, sd, sd)) < s_p)
    image = np.zeros((img, img), bool)
    sw_s, sw_w, sw_pix = [], [], []
    for k in range(K):
        for p in range(sd):
            for q in range(sd):
                for a in range(tw):
                    for bb in range(tw):
                        i, jj = p + a, q + bb
                        if i < img and jj < img:
                            sw_s.append(nW + (k * sd + p) * sd + q)
                            sw_w.append((k * tw + a) * tw + bb)
                            sw_pix.append(i * img + jj)
                            if gtS[k, p, q] and gtW[k, a, bb]:
                                image[i, jj] = True
    nSW = len(sw_s)
    V = nW + nS + nSW + img * img
    sw0 = nW + nS
    x0 = sw0 + nSW
    ev = np.zeros((V, 2), np.float32)
    ev[: nW + nS, 1] = lam
    ev[x0:, 1] = np.where(image.reshape(-1), clamp, -clamp)
    sw_s = np.asarray(sw_s, np.int64)
    sw_w = np.asarray(sw_w, np.int64)
    sw_pix = np.asarray(sw_pix, np.int64)
    # AND factors: (S, W, SW)
    and_edges = np.stack([sw_s, sw_w, sw0 + np.arange(nSW)], 1).reshape(-1)
    # OR factors: parents grouped per pixel (stable, creation order), child X
    order = np.argsort(sw_pix, kind="stable")
    counts = np.bincount(sw_pix, minlength=img * img)
    or_edges, or_off = [], [0]
    pos = 0
    for pix in range(img * img):
        c = counts[pix]
        par = sw0 + order[pos:pos + c]
        pos += c
        or_edges.append(np.concatenate([par, [x0 + pix]]))
        or_off.append(or_off[-1] + c + 1)
    or_edges = np.concatenate(or_edges)
    F = nSW + img * img
    fe_off = np.concatenate([np.arange(nSW + 1, dtype=np.int64) * 3,
                             3 * nSW + np.asarray(or_off[1:], np.int64)])
    kind = np.concatenate([np.full(nSW, AND, np.int32), np.full(img * img, OR, np.int32)])
    return GraphSpec(
        var_num_states=np.full(V, 2, np.int32), evidence=ev.reshape(-1),
        factor_kind=kind, factor_edge_off=fe_off,
        edge_var=np.concatenate([and_edges, or_edges]),
        factor_cfg_table=np.full(F, -1, np.int32),
        cfg_table_num_cfgs=np.zeros(0, np.int32), cfg_table_arity=np.zeros(0, np.int32),
        cfg_table_off=np.zeros(1, np.int64), cfg_table_states=np.zeros(0, np.int32),
        logpot_off=np.zeros(F + 1, np.int64), log_potentials=np.zeros(0, np.float32),
        name="deconv", meta={"seed": seed, "image_density": float(image.mean()),
                             "gt_active": int(gtS.sum()), "nW": nW, "nS": nS,
                             "nSW": nSW, "nX": img * img},
    )


# ---------------------------------------------------------------------------
# small random graphs for tests
# ---------------------------------------------------------------------------
def _general_graph(nstates, ev, factors, name, meta=None):
    """Assemble a GraphSpec from a list of factor records.

    Each record is a dict with ``kind`` (ENUM/OR/AND), ``vars`` and, for
    enumeration factors, ``logpot`` and optionally ``configs`` (explicit table,
    shape (num_cfgs, arity)); without ``configs`` the table is dense."""
    nstates = np.asarray(nstates, np.int32)
    tables = {}  # key -> table id
    t_ncfg, t_ar, t_states, t_off = [], [], [], [0]
    kind, fe_off, evar, ftab, lp_off, lps = [], [0], [], [], [0], []
    for fr in factors:
        k = fr["kind"]
        vs = list(fr["vars"])
        kind.append(k)
        evar.extend(vs)
        fe_off.append(len(evar))
        if k == ENUM:
            cfg = fr.get("configs")
            if cfg is None:
                key = ("dense", len(vs))
                if key not in tables:
                    tables[key] = len(t_ncfg)
                    t_ncfg.append(0)
                    t_ar.append(len(vs))
                    t_off.append(t_off[-1])
            else:
                cfg = np.asarray(cfg, np.int32)
                key = ("explicit", cfg.tobytes(), cfg.shape)
                if key not in tables:
                    tables[key] = len(t_ncfg)
                    t_ncfg.append(cfg.shape[0])
                    t_ar.append(cfg.shape[1])
                    t_states.append(cfg.reshape(-1))
                    t_off.append(t_off[-1] + cfg.size)
            ftab.append(tables[key])
            lp = np.asarray(fr["logpot"], np.float32).reshape(-1)
            lps.append(lp)
            lp_off.append(lp_off[-1] + lp.size)
        else:
            ftab.append(-1)
            lp_off.append(lp_off[-1])
    return GraphSpec(
        var_num_states=nstates, evidence=ev, factor_kind=np.asarray(kind, np.int32),
        factor_edge_off=np.asarray(fe_off, np.int64), edge_var=np.asarray(evar, np.int32),
        factor_cfg_table=np.asarray(ftab, np.int32),
        cfg_table_num_cfgs=np.asarray(t_ncfg, np.int32),
        cfg_table_arity=np.asarray(t_ar, np.int32),
        cfg_table_off=np.asarray(t_off, np.int64),
        cfg_table_states=(np.concatenate(t_states) if t_states else np.zeros(0, np.int32)),
        logpot_off=np.asarray(lp_off, np.int64),
        log_potentials=(np.concatenate(lps) if lps else np.zeros(0, np.float32)),
        name=name, meta=meta or {},
    )


def _random_explicit_configs(rng, ns, frac=0.6):
    """A random subset of the joint states of a factor that still covers every
    (slot, state) pair at least once."""
    full = np.stack(np.meshgrid(*[np.arange(n) for n in ns], indexing="ij"), -1).reshape(-1, len(ns))
    while True:
        keep = rng.random(full.shape[0]) < frac
        sub = full[keep]
        if sub.shape[0] and all(len(np.unique(sub[:, j])) == ns[j] for j in range(len(ns))):
            return sub


def random_factor_graph(seed: int, num_vars: int, max_states: int = 4, tree: bool = True,
                        extra_factors: int = 0, max_arity: int = 3, logical_frac: float = 0.0,
                        explicit_frac: float = 0.3, ev_sd: float = 1.0, lp_sd: float = 1.0,
                        name: str = "random") -> GraphSpec:
    """Random factor graph.  With ``tree`` the variable-factor graph is a tree:
    factors are added one by one, each joining one already-connected variable
    with 1..max_arity-1 new ones.  ``extra_factors`` then adds factors over
    random existing variables, which closes loops.  A fraction of factors are
    OR/AND (their variables become binary), the rest are enumeration factors
    with dense or explicit tables."""
    rng = np.random.default_rng(seed)
    nst = rng.integers(2, max_states + 1, size=num_vars).astype(np.int32)
    factors = []
    connected = [0]
    free = list(range(1, num_vars))
    plans = []
    while free:
        k = int(rng.integers(1, max_arity)) if max_arity > 1 else 1
        k = min(k, len(free))
        anchor = int(rng.choice(connected))
        new = [free.pop(0) for _ in range(k)]
        connected.extend(new)
        plans.append([anchor] + new)
    for _ in range(extra_factors):
        k = int(rng.integers(2, max_arity + 1))
        k = min(k, num_vars)
        plans.append([int(x) for x in rng.choice(num_vars, size=k, replace=False)])
    logical = rng.random(len(plans)) < logical_frac
    for f, vs in enumerate(plans):
        if logical[f]:
            for v in vs:
                nst[v] = 2
    for f, vs in enumerate(plans):
        if logical[f]:
            factors.append({"kind": OR if rng.random() < 0.5 else AND,
                            "vars": vs[1:] + vs[:1] if len(vs) > 1 else vs})
    # enumeration factors after the state counts are final
    out = []
    li = 0
    for f, vs in enumerate(plans):
        if logical[f]:
            out.append(factors[li])
            li += 1
            continue
        ns = [int(nst[v]) for v in vs]
        if rng.random() < explicit_frac:
            cfg = _random_explicit_configs(rng, ns)
            out.append({"kind": ENUM, "vars": vs, "configs": cfg,
                        "logpot": rng.normal(0, lp_sd, size=cfg.shape[0])})
        else:
            out.append({"kind": ENUM, "vars": vs,
                        "logpot": rng.normal(0, lp_sd, size=int(np.prod(ns)))})
    ev = rng.normal(0.0, ev_sd, size=int(nst.sum())).astype(np.float32)
    return _general_graph(nst, ev, out, name, {"seed": seed, "tree": tree and extra_factors == 0})


def chain(seed: int, length: int, n: int = 3, ev_sd: float = 1.0, lp_sd: float = 1.0) -> GraphSpec:
    """Chain of ``length`` variables with n states and dense pairwise factors."""
    rng = np.random.default_rng(seed)
    ev = rng.normal(0, ev_sd, size=length * n).astype(np.float32)
    pairs = np.stack([np.arange(length - 1), np.arange(1, length)], 1)
    tab = rng.normal(0, lp_sd, size=(length - 1, n * n))
    return _pairwise_graph(np.full(length, n, np.int32), ev, pairs, tab, f"chain{length}")


def single_logical(seed: int, kind: int, num_parents: int, ev_sd: float = 1.5) -> GraphSpec:
    """One OR/AND factor over ``num_parents`` parents and a child, random evidence."""
    rng = np.random.default_rng(seed)
    V = num_parents + 1
    ev = rng.normal(0, ev_sd, size=V * 2).astype(np.float32)
    return _general_graph(np.full(V, 2, np.int32), ev,
                          [{"kind": kind, "vars": list(range(V))}], f"logic{kind}_{num_parents}")


def single_enum(seed: int, nstates, explicit: bool = False, ev_sd: float = 1.0,
                lp_sd: float = 1.0) -> GraphSpec:
    """One enumeration factor over variables with the given state counts."""
    rng = np.random.default_rng(seed)
    ns = [int(x) for x in nstates]
    ev = rng.normal(0, ev_sd, size=sum(ns)).astype(np.float32)
    if explicit:
        cfg = _random_explicit_configs(rng, ns)
        fr = {"kind": ENUM, "vars": list(range(len(ns))), "configs": cfg,
              "logpot": rng.normal(0, lp_sd, size=cfg.shape[0])}
    else:
        fr = {"kind": ENUM, "vars": list(range(len(ns))),
              "logpot": rng.normal(0, lp_sd, size=int(np.prod(ns)))}
    return _general_graph(np.asarray(ns, np.int32), ev, [fr], "enum1")


def random_rbm_small(seed: int, nv: int = 15, nh: int = 15, w_sd: float = 1.0,
                     b_sd: float = 0.5) -> GraphSpec:
    """Small RBM for the MAP-quality protocol (ground truth by enumeration)."""
    return rbm(nv, nh, seed=seed, w_sd=w_sd, b_sd=b_sd)


def disjoint_union(graphs) -> GraphSpec:
    """Disjoint union of factor graphs (variables, factors and tables renumbered)."""
    parts = {k: [] for k in ARRAY_FIELDS}
    v_base = e_base = t_base = lp_base = ts_base = 0
    fe = [np.zeros(1, np.int64)]
    lpo = [np.zeros(1, np.int64)]
    cto = [np.zeros(1, np.int64)]
    for g in graphs:
        parts["var_num_states"].append(g.var_num_states)
        parts["evidence"].append(g.evidence)
        parts["factor_kind"].append(g.factor_kind)
        fe.append(g.factor_edge_off[1:] + e_base)
        parts["edge_var"].append(g.edge_var + v_base)
        parts["factor_cfg_table"].append(np.where(g.factor_cfg_table >= 0,
                                                  g.factor_cfg_table + t_base, -1))
        parts["cfg_table_num_cfgs"].append(g.cfg_table_num_cfgs)
        parts["cfg_table_arity"].append(g.cfg_table_arity)
        cto.append(g.cfg_table_off[1:] + ts_base)
        parts["cfg_table_states"].append(g.cfg_table_states)
        lpo.append(g.logpot_off[1:] + lp_base)
        parts["log_potentials"].append(g.log_potentials)
        v_base += g.num_vars
        e_base += g.num_edges
        t_base += g.cfg_table_num_cfgs.shape[0]
        ts_base += g.cfg_table_states.shape[0]
        lp_base += g.num_logpots
    out = {k: np.concatenate(v) if v else np.zeros(0) for k, v in parts.items()
           if k not in ("factor_edge_off", "logpot_off", "cfg_table_off")}
    out["factor_edge_off"] = np.concatenate(fe)
    out["logpot_off"] = np.concatenate(lpo)
    out["cfg_table_off"] = np.concatenate(cto)
    return GraphSpec(name="union", **out)


# ---------------------------------------------------------------------------
# served stream
# ---------------------------------------------------------------------------
def served_requests(num: int = 512, seed: int = 5, min_side: int = 16, max_side: int = 256,
                    min_states: int = 2, max_states: int = 8, backward_count: int = 51):
    """Request mix for the serving loop: square Potts grids whose side is
    log-uniform in [min_side, max_side] and whose state count is uniform in
    [min_states, max_states]; the graph of request i is drawn from seed
    ``seed + i`` as ``potts_grid``.  A seeded choice of ``backward_count``
    requests also carry a loss-gradient vector c ~ N(0,1) over their
    variable-states (loss = sum c * q).  Returns a list of dicts holding the
    shape parameters; graphs are built on demand by ``request_graph``."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(math.log(min_side), math.log(max_side), size=num))).astype(int)
    states = rng.integers(min_states, max_states + 1, size=num)
    bwd = np.zeros(num, bool)
    bwd[rng.choice(num, size=min(backward_count, num), replace=False)] = True
    return [{"id": i, "L": int(sides[i]), "n": int(states[i]), "seed": seed + 1000 + i,
             "backward": bool(bwd[i])} for i in range(num)]


def request_graph(req) -> GraphSpec:
    return potts_grid(req["L"], req["n"], seed=req["seed"])


def request_loss_coeffs(req) -> np.ndarray:
    rng = np.random.default_rng(req["seed"] + 7)
    return rng.normal(0, 1, size=req["L"] * req["L"] * req["n"]).astype(np.float32)


def poisson_arrivals(num: int, qps: float, seed: int = 5) -> np.ndarray:
    """Arrival offsets in seconds for a Poisson process of rate ``qps``."""
    rng = np.random.default_rng(seed + 99)
    return np.cumsum(rng.exponential(1.0 / qps, size=num))
