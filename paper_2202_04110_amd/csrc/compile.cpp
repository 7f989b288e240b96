// Validation of a factor-graph description and its compilation into the
// panel layout used by the kernels (see lbp_internal.h).
//
// The flat-array idea is the paper's (Sec. "A fully flat array-based LBP
// implementation": messages in flat arrays, global indices of variable states
// and valid configurations computed once); the panel layout, the shape
// classes and the tile tables are this library's own.
#include "compile.h"

#include <algorithm>
#include <climits>
#include <cstring>
#include <cmath>
#include <map>
#include <string>
#include <tuple>
#include <vector>

namespace lbp {
namespace {

int bad(std::string *err, const std::string &msg, int code = LBP_E_INVALID) {
    *err = msg;
    return code;
}

// Index of the first infinite or NaN element, or -1: an exponent-bits test
// over blocks (branch-free, so it vectorises), then a scan of a hit block.
int64_t first_nonfinite(const float *x, int64_t n) {
    constexpr int64_t B = 4096;
    for (int64_t b = 0; b < n; b += B) {
        const int64_t e = std::min(n, b + B);
        uint32_t hit = 0;
        for (int64_t i = b; i < e; ++i) {
            uint32_t u;
            std::memcpy(&u, x + i, sizeof u);
            hit |= (uint32_t)((u & 0x7f800000u) == 0x7f800000u);
        }
        if (hit)
            for (int64_t i = b; i < e; ++i)
                if (!std::isfinite(x[i])) return i;
    }
    return -1;
}

std::string at(const char *what, int64_t i) { return std::string(what) + "[" + std::to_string(i) + "]"; }

bool monotone_from_zero(const int64_t *off, int64_t n) {
    if (off[0] != 0) return false;
    for (int64_t i = 0; i < n; ++i)
        if (off[i + 1] < off[i]) return false;
    return true;
}

// Whether an enumeration factor with these slot state counts uses the dense
// pairwise fast path.
bool pair_fast(bool dense, int32_t arity, const int32_t *ns) {
    return dense && arity == 2 && ns[0] <= kPairStatesMax && ns[1] <= kPairStatesMax;
}

// Internal variable order.  A logical factor with more edges than a lane
// tile holds is gathered by one wavefront, which reads the beliefs of all
// its parents (every edge but the last); parents with at most two edges are
// renumbered consecutively in the order those factors list them, into the
// positions they held (every other variable keeps its id), so that the
// gather reads consecutive lanes of few panels.  order[i] = the caller's id
// of internal id i; false (and order empty) when no variable moves.
bool internal_order(const lbp_graph_desc *d, std::vector<int32_t> *order) {
    const int64_t V = d->num_vars, F = d->num_factors, E = V > 0 ? d->factor_edge_off[F] : 0;
    auto wide = [&](int64_t f) {
        return d->factor_kind[f] != LBP_FACTOR_ENUM &&
               d->factor_edge_off[f + 1] - d->factor_edge_off[f] > kLogLaneArityMax;
    };
    bool any = false;
    for (int64_t f = 0; f < F && !any; ++f) any = wide(f);
    if (!any) return false;
    std::vector<int32_t> deg(V, 0);
    for (int64_t e = 0; e < E; ++e) ++deg[d->edge_var[e]];
    std::vector<char> taken(V, 0);
    std::vector<int32_t> seq;
    for (int64_t f = 0; f < F; ++f) {
        if (!wide(f)) continue;
        for (int64_t e = d->factor_edge_off[f]; e + 1 < d->factor_edge_off[f + 1]; ++e) {
            const int32_t v = d->edge_var[e];
            if (deg[v] <= 2 && !taken[v]) {
                taken[v] = 1;
                seq.push_back(v);
            }
        }
    }
    std::vector<int32_t> pos(seq);
    std::sort(pos.begin(), pos.end());
    order->resize(V);
    for (int64_t v = 0; v < V; ++v) (*order)[v] = (int32_t)v;
    bool moved = false;
    for (size_t i = 0; i < seq.size(); ++i) {
        (*order)[pos[i]] = seq[i];
        moved = moved || pos[i] != seq[i];
    }
    if (!moved) order->clear();
    return moved;
}

}  // namespace

int validate_desc(const lbp_graph_desc *d, int64_t sizes[6], std::string *err, bool scan_potentials) {
    if (!d) return bad(err, "graph description is NULL");
    const int64_t V = d->num_vars, F = d->num_factors, NT = d->num_cfg_tables;
    if (V < 0 || F < 0 || NT < 0) return bad(err, "negative num_vars, num_factors or num_cfg_tables");
    if (V > 0 && !d->var_num_states) return bad(err, "var_num_states is NULL");
    if (!d->factor_edge_off || !d->logpot_off) return bad(err, "factor_edge_off or logpot_off is NULL");
    if (F > 0 && (!d->factor_kind || !d->factor_cfg_table))
        return bad(err, "factor_kind or factor_cfg_table is NULL");
    if (NT > 0 && (!d->cfg_table_num_cfgs || !d->cfg_table_arity || !d->cfg_table_off))
        return bad(err, "configuration table arrays are NULL");

    int64_t VS = 0;
    for (int64_t v = 0; v < V; ++v) {
        int32_t n = d->var_num_states[v];
        if (n < 2 || n > kMaxStates)
            return bad(err, at("var_num_states", v) + " = " + std::to_string(n) + " outside [2, 64]");
        VS += n;
    }
    if (d->evidence) {
        const int64_t i = first_nonfinite(d->evidence, VS);
        if (i >= 0) return bad(err, at("evidence", i) + " is not finite");
    }

    if (!monotone_from_zero(d->factor_edge_off, F))
        return bad(err, "factor_edge_off must start at 0 and be non-decreasing");
    const int64_t E = d->factor_edge_off[F];
    if (E > INT32_MAX) return bad(err, "more than 2^31-1 edges", LBP_E_UNSUPPORTED);
    if (E > 0 && !d->edge_var) return bad(err, "edge_var is NULL");
    for (int64_t e = 0; e < E; ++e)
        if (d->edge_var[e] < 0 || d->edge_var[e] >= V)
            return bad(err, at("edge_var", e) + " out of range");

    if (!monotone_from_zero(d->logpot_off, F))
        return bad(err, "logpot_off must start at 0 and be non-decreasing");
    const int64_t Tn = d->logpot_off[F];
    if (Tn > 0 && !d->log_potentials) return bad(err, "log_potentials is NULL");
    if (scan_potentials) {
        const int64_t i = first_nonfinite(d->log_potentials, Tn);
        if (i >= 0) return bad(err, at("log_potentials", i) + " is not finite");
    }

    if (NT > 0) {
        if (!monotone_from_zero(d->cfg_table_off, NT))
            return bad(err, "cfg_table_off must start at 0 and be non-decreasing");
        if (d->cfg_table_off[NT] > 0 && !d->cfg_table_states) return bad(err, "cfg_table_states is NULL");
        for (int64_t t = 0; t < NT; ++t) {
            int64_t a = d->cfg_table_arity[t], c = d->cfg_table_num_cfgs[t];
            int64_t len = d->cfg_table_off[t + 1] - d->cfg_table_off[t];
            if (a < 1) return bad(err, at("cfg_table_arity", t) + " < 1");
            if (c < 0) return bad(err, at("cfg_table_num_cfgs", t) + " < 0");
            if (len != c * a) return bad(err, "table " + std::to_string(t) + " holds " +
                                                 std::to_string(len) + " states, expected num_cfgs*arity");
        }
    }

    // explicit tables checked once per (table, slot state counts)
    std::map<std::vector<int32_t>, int> checked;
    for (int64_t f = 0; f < F; ++f) {
        const int64_t e0 = d->factor_edge_off[f];
        const int64_t k = d->factor_edge_off[f + 1] - e0;
        const int64_t nlp = d->logpot_off[f + 1] - d->logpot_off[f];
        const int32_t kind = d->factor_kind[f];
        if (kind == LBP_FACTOR_ENUM) {
            if (k < 1) return bad(err, "enumeration factor " + std::to_string(f) + " has no edge");
            int32_t t = d->factor_cfg_table[f];
            if (t < 0 || t >= NT) return bad(err, at("factor_cfg_table", f) + " out of range");
            if (d->cfg_table_arity[t] != k)
                return bad(err, "factor " + std::to_string(f) + " has arity " + std::to_string(k) +
                                    " but its table has arity " + std::to_string(d->cfg_table_arity[t]));
            int64_t nsum = 0;
            int32_t ns2[2] = {0, 0};
            for (int64_t j = 0; j < k; ++j) {
                const int32_t n = d->var_num_states[d->edge_var[e0 + j]];
                if (j < 2) ns2[j] = n;
                nsum += n;
            }
            const bool dense = d->cfg_table_num_cfgs[t] == 0;
            int64_t ncfg;
            if (dense) {
                ncfg = 1;
                for (int64_t j = 0; j < k; ++j) {
                    ncfg *= d->var_num_states[d->edge_var[e0 + j]];
                    if (ncfg > INT32_MAX) return bad(err, "dense table of factor " + std::to_string(f) +
                                                              " is too large", LBP_E_UNSUPPORTED);
                }
            } else {
                ncfg = d->cfg_table_num_cfgs[t];
                std::vector<int32_t> ns(k);
                for (int64_t j = 0; j < k; ++j) ns[j] = d->var_num_states[d->edge_var[e0 + j]];
                std::vector<int32_t> key(ns);
                key.push_back(t);
                if (!checked.count(key)) {
                    std::vector<std::vector<char>> cov(k);
                    for (int64_t j = 0; j < k; ++j) cov[j].assign(ns[j], 0);
                    const int32_t *st = d->cfg_table_states + d->cfg_table_off[t];
                    for (int64_t c = 0; c < ncfg; ++c)
                        for (int64_t j = 0; j < k; ++j) {
                            int32_t s = st[c * k + j];
                            if (s < 0 || s >= ns[j])
                                return bad(err, "table " + std::to_string(t) + " config " + std::to_string(c) +
                                                    " slot " + std::to_string(j) + " state out of range for factor " +
                                                    std::to_string(f));
                            cov[j][s] = 1;
                        }
                    for (int64_t j = 0; j < k; ++j)
                        for (int32_t s = 0; s < ns[j]; ++s)
                            if (!cov[j][s])
                                return bad(err, "factor " + std::to_string(f) + ": no configuration has slot " +
                                                    std::to_string(j) + " in state " + std::to_string(s));
                    checked[key] = 1;
                }
            }
            if (nlp != ncfg)
                return bad(err, "factor " + std::to_string(f) + " has " + std::to_string(nlp) +
                                    " log-potentials, its table " + std::to_string(ncfg) + " configurations");
            if (!pair_fast(dense, (int32_t)k, ns2) &&
                (k > kGenArityMax || ncfg > kGenCfgMax || nsum > kGenRowsMax))
                return bad(err, "enumeration factor " + std::to_string(f) +
                                    " exceeds the generic kernel limits (arity <= 8, <= 4096 configurations, "
                                    "<= 64 summed slot states)", LBP_E_UNSUPPORTED);
        } else if (kind == LBP_FACTOR_OR || kind == LBP_FACTOR_AND) {
            if (k < 2) return bad(err, "logical factor " + std::to_string(f) + " needs a parent and a child");
            if (k > kLogWaveArityMax)
                return bad(err, "logical factor " + std::to_string(f) + " has more than 1024 edges",
                           LBP_E_UNSUPPORTED);
            for (int64_t j = 0; j < k; ++j)
                if (d->var_num_states[d->edge_var[e0 + j]] != 2)
                    return bad(err, "logical factor " + std::to_string(f) + " touches a non-binary variable");
            if (nlp != 0) return bad(err, "logical factor " + std::to_string(f) + " has log-potentials");
        } else {
            return bad(err, at("factor_kind", f) + " is not 0, 1 or 2");
        }
    }
    int64_t ES = 0;
    for (int64_t e = 0; e < E; ++e) ES += d->var_num_states[d->edge_var[e]];
    if (sizes) {
        sizes[0] = V; sizes[1] = VS; sizes[2] = F; sizes[3] = E; sizes[4] = ES; sizes[5] = Tn;
    }
    return LBP_OK;
}

int compile_desc(const lbp_graph_desc *d_in, HostLayout *L, std::string *err, bool fill) {
    int64_t sz[6];
    // the potentials are checked for NaN and infinity while they are copied
    // into their panels (every one of them is), not in a pass of their own
    int rc = validate_desc(d_in, sz, err, false);
    if (rc != LBP_OK) return rc;
    L->V = sz[0]; L->VS = sz[1]; L->F = sz[2]; L->E = sz[3]; L->ES = sz[4]; L->Tn = sz[5];
    const int64_t V = L->V, F = L->F, E = L->E;

    // The layout is built over the variables in internal order, from a copy
    // of the description whose edges name internal ids (factors keep theirs).
    const lbp_graph_desc *d = d_in;
    lbp_graph_desc pd;
    std::vector<int32_t> p_nst, p_evar;
    L->vext.clear();
    if (internal_order(d_in, &L->vext)) {
        std::vector<int32_t> inv(V);
        for (int64_t i = 0; i < V; ++i) inv[L->vext[i]] = (int32_t)i;
        p_nst.resize(V);
        for (int64_t i = 0; i < V; ++i) p_nst[i] = d_in->var_num_states[L->vext[i]];
        p_evar.resize(E);
        for (int64_t e = 0; e < E; ++e) p_evar[e] = inv[d_in->edge_var[e]];
        pd = *d_in;
        pd.var_num_states = p_nst.data();
        pd.edge_var = p_evar.data();
        pd.evidence = nullptr;  // read through vs_off from the caller's description only
        d = &pd;
    }

    L->vs_off.assign(V + 1, 0);
    L->vn.assign(V, 0);
    for (int64_t v = 0; v < V; ++v) {
        L->vn[v] = d->var_num_states[v];
        L->vs_off[v + 1] = L->vs_off[v] + L->vn[v];
    }
    if (!L->vext.empty()) {  // offsets in the caller's flat order
        std::vector<int64_t> ext(V + 1, 0);
        for (int64_t v = 0; v < V; ++v) ext[v + 1] = ext[v] + d_in->var_num_states[v];
        for (int64_t i = 0; i < V; ++i) L->vs_off[i] = ext[L->vext[i]];
        L->vs_off[V] = ext[V];
    }
    L->es_off.assign(E + 1, 0);
    for (int64_t e = 0; e < E; ++e) L->es_off[e + 1] = L->es_off[e] + L->vn[d->edge_var[e]];
    L->lp_off.assign(d->logpot_off, d->logpot_off + F + 1);

    // ---------------------------------------------------------- variable tiles
    const int64_t nvt = (V + kLanes - 1) / kLanes;
    std::vector<int32_t> vaddr(V);
    L->vtile.resize(nvt);
    int64_t VB = 0;
    for (int64_t t = 0; t < nvt; ++t) {
        int32_t nt = 2;
        for (int64_t v = t * kLanes; v < std::min<int64_t>(V, (t + 1) * kLanes); ++v) nt = std::max(nt, L->vn[v]);
        L->vtile[t].b_off = (int32_t)VB;
        L->vtile[t].n = nt;
        for (int64_t v = t * kLanes; v < std::min<int64_t>(V, (t + 1) * kLanes); ++v)
            vaddr[v] = (int32_t)(VB + (v - t * kLanes));
        VB += (int64_t)kLanes * nt;
        if (VB >= INT32_MAX) return bad(err, "belief array exceeds 2^31 floats", LBP_E_UNSUPPORTED);
    }
    // a spare panel that idle lanes of partly filled factor tiles point at
    const int32_t b_zero = (int32_t)VB;
    VB += (int64_t)kLanes * kMaxStates;
    L->VB = VB;
    std::vector<int32_t> tile_fac;  // factor of each (tile, lane) with a potential panel, -1 otherwise
    // the tiles' rows hold every edge once plus idle lanes: room for the
    // edges and a few partial tiles, so the arrays rarely grow by copying
    L->fvb.reserve((size_t)E + 64 * kLanes);
    L->fvar.reserve((size_t)E + 64 * kLanes);
    L->ftile.reserve((size_t)F / kLanes + 64);
    tile_fac.reserve((size_t)F + 64 * kLanes);
    auto add_vb_rows = [&](int32_t rows) {
        tile_fac.resize((L->ftile.size() + 1) * kLanes, -1);
        const size_t base = L->fvb.size();
        L->fvb.resize(base + (size_t)rows * kLanes);
        L->fvar.resize(base + (size_t)rows * kLanes, -1);
        for (int32_t r = 0; r < rows; ++r)
            for (int32_t l = 0; l < kLanes; ++l) L->fvb[base + (size_t)r * kLanes + l] = b_zero + l;
    };

    // variable -> edges, increasing edge order
    std::vector<int64_t> adj_off(V + 1, 0), adj(E);
    for (int64_t e = 0; e < E; ++e) adj_off[d->edge_var[e] + 1]++;
    for (int64_t v = 0; v < V; ++v) adj_off[v + 1] += adj_off[v];
    {
        std::vector<int64_t> fill(adj_off.begin(), adj_off.end() - 1);
        for (int64_t e = 0; e < E; ++e) adj[fill[d->edge_var[e]]++] = e;
    }

    // ---------------------------------------------------------- factor classes
    // key: (tile kind, a, b, table, slot state counts)
    typedef std::tuple<int32_t, int32_t, int32_t, int32_t, std::vector<int32_t>> Key;
    std::map<Key, int32_t> class_of;
    std::vector<Key> class_key;
    std::vector<std::vector<int32_t>> class_facs;
    std::vector<int32_t> fclass(F);
    // Small integer codes for the common shapes avoid building a key per
    // factor: dense pairwise (na, nb), lane logical (arity, AND), wide logical
    // (chunk bucket).  Generic classes use the full key.
    std::vector<int32_t> fast_class(2 * 65 * 65 + 64, -1);
    auto fast_code = [&](int32_t kind, int32_t a, int32_t b) -> int32_t {
        if (kind == TK_PAIR) return a * 65 + b;
        if (kind == TK_LOGL) return 65 * 65 + a * 2 + b;
        return 65 * 65 + 2 * (kLogLaneArityMax + 1) + a;  // TK_LOGW: a = chunk bucket <= 16
    };
    for (int64_t f = 0; f < F; ++f) {
        const int64_t e0 = d->factor_edge_off[f];
        const int32_t k = (int32_t)(d->factor_edge_off[f + 1] - e0);
        int32_t kind, a = 0, b = 0;
        bool fast = true;
        if (d->factor_kind[f] == LBP_FACTOR_ENUM) {
            const int32_t t = d->factor_cfg_table[f];
            const bool dense = d->cfg_table_num_cfgs[t] == 0;
            int32_t ns2[2] = {k > 0 ? L->vn[d->edge_var[e0]] : 0, k > 1 ? L->vn[d->edge_var[e0 + 1]] : 0};
            if (pair_fast(dense, k, ns2)) {
                kind = TK_PAIR;
                a = ns2[0];
                b = ns2[1];
            } else {
                kind = TK_GEN;
                fast = false;
            }
        } else if (k <= kLogLaneArityMax) {
            kind = TK_LOGL;
            a = k;
            b = d->factor_kind[f] == LBP_FACTOR_AND;
        } else {  // one tile per factor
            kind = TK_LOGW;
            a = chunk_bucket((k + kLanes - 1) / kLanes);
        }
        int32_t c;
        if (fast) {
            int32_t &slot = fast_class[fast_code(kind, a, b)];
            if (slot < 0) {
                slot = (int32_t)class_key.size();
                class_key.push_back(Key(kind, a, b, -1, std::vector<int32_t>()));
                class_facs.emplace_back();
            }
            c = slot;
        } else {
            std::vector<int32_t> ns(k);
            for (int32_t j = 0; j < k; ++j) ns[j] = L->vn[d->edge_var[e0 + j]];
            const int32_t t = d->factor_cfg_table[f];
            Key key(TK_GEN, k, 0, d->cfg_table_num_cfgs[t] == 0 ? -1 : t, ns);
            auto it = class_of.find(key);
            if (it == class_of.end()) {
                c = (int32_t)class_key.size();
                class_of[key] = c;
                class_key.push_back(key);
                class_facs.emplace_back();
            } else {
                c = it->second;
            }
        }
        fclass[f] = c;
    }
    {  // members in factor order, each class sized once
        std::vector<size_t> cnt(class_key.size(), 0);
        for (int64_t f = 0; f < F; ++f) ++cnt[fclass[f]];
        for (size_t c = 0; c < class_key.size(); ++c) class_facs[c].reserve(cnt[c]);
        for (int64_t f = 0; f < F; ++f) class_facs[fclass[f]].push_back((int32_t)f);
    }

    L->edge_maddr.assign(E, 0);
    L->fac_phi.assign(F, -1);
    int64_t M = 0, P = 0;
    auto check = [&](int64_t x, const char *what) {
        return x < INT32_MAX - 4096 ? LBP_OK : bad(err, std::string(what) + " exceeds 2^31 floats", LBP_E_UNSUPPORTED);
    };
    std::vector<std::pair<int64_t, float>> phi_fill;  // filled after sizing
    // Within a lane-per-factor class, order factors by the 64-variable block
    // of their first variable (then by index): a tile's factors then touch
    // few variable tiles, which keeps belief reads local.  Tile membership
    // does not change any factor's arithmetic.
    // (a stable counting sort on the block index when the class is large
    // against the number of blocks, a comparison sort otherwise: same order)
    const int64_t nblk = (V + kLanes - 1) / kLanes;
    std::vector<int32_t> blk_start, sorted;
    for (size_t c = 0; c < class_key.size(); ++c) {
        if (std::get<0>(class_key[c]) == TK_LOGW) continue;
        std::vector<int32_t> &fl = class_facs[c];
        auto key = [&](int32_t f) { return d->edge_var[d->factor_edge_off[f]] / kLanes; };
        if ((int64_t)fl.size() >= nblk / 4) {
            blk_start.assign(nblk + 1, 0);
            for (int32_t f : fl) ++blk_start[key(f) + 1];
            for (int64_t b = 0; b < nblk; ++b) blk_start[b + 1] += blk_start[b];
            sorted.resize(fl.size());
            for (int32_t f : fl) sorted[blk_start[key(f)]++] = f;
            fl.swap(sorted);
        } else {
            std::stable_sort(fl.begin(), fl.end(), [&](int32_t x, int32_t y) { return key(x) < key(y); });
        }
        if (std::get<0>(class_key[c]) == TK_LOGL && !L->vext.empty()) {
            // renumbered variables (wide logical factors' parents): within a
            // block, by the internal id of the child, so a tile's children
            // are consecutive parents of a few wide factors while its first
            // variables stay in one block (measured on the deconvolution
            // graph against ordering by the child alone: within 2% either
            // way, this one ahead with the tuned launch shapes)
            auto child = [&](int32_t f) { return d->edge_var[d->factor_edge_off[f + 1] - 1]; };
            for (size_t i = 0; i < fl.size();) {
                size_t j = i;
                while (j < fl.size() && key(fl[j]) == key(fl[i])) ++j;
                std::stable_sort(fl.begin() + (int64_t)i, fl.begin() + (int64_t)j,
                                 [&](int32_t x, int32_t y) { return child(x) < child(y); });
                i = j;
            }
        }
        if (std::get<0>(class_key[c]) != TK_PAIR) continue;
        // pairwise factors that all join two block-path variables (a dense
        // bipartite layer): ordered by the 16-variable block of the second
        // variable, then the first, so a tile holds 4 x 16 factors and a run
        // of tiles (the share of one XCD in the factor launch) covers a range
        // of second variables, the range the column groups of those
        // variables read from on the same XCD in the variable launch
        {
            auto var0 = [&](int32_t f) { return (int64_t)d->edge_var[d->factor_edge_off[f]]; };
            auto var1 = [&](int32_t f) { return (int64_t)d->edge_var[d->factor_edge_off[f] + 1]; };
            bool layer = !fl.empty();
            for (size_t i = 0; i < fl.size() && layer; ++i)
                layer = adj_off[var0(fl[i]) + 1] - adj_off[var0(fl[i])] > kMidDegMax &&
                        adj_off[var1(fl[i]) + 1] - adj_off[var1(fl[i])] > kMidDegMax;
            if (layer) {
                // two stable counting passes: by first variable, then by
                // the second variable's block
                auto pass = [&](auto bucket, int64_t nb) {
                    std::vector<int64_t> at(nb + 1, 0);
                    for (int32_t f : fl) ++at[bucket(f) + 1];
                    for (int64_t b = 0; b < nb; ++b) at[b + 1] += at[b];
                    sorted.resize(fl.size());
                    for (int32_t f : fl) sorted[at[bucket(f)]++] = f;
                    fl.swap(sorted);
                };
                pass(var0, V);
                pass([&](int32_t f) { return var1(f) / 16; }, V / 16 + 1);
                continue;
            }
        }
        // pairwise: inside a block whose factors join their two variables at
        // no more than four distinct offsets (a grid: horizontal and vertical
        // neighbours), factors with the same offset together, each group in
        // its existing order; other blocks keep their order
        auto delta = [&](int32_t f) {
            const int64_t e0 = d->factor_edge_off[f];
            return (int64_t)d->edge_var[e0 + 1] - d->edge_var[e0];
        };
        std::vector<int32_t> part;
        for (size_t i = 0; i < fl.size();) {
            size_t j = i;
            while (j < fl.size() && key(fl[j]) == key(fl[i])) ++j;
            int64_t seen[4];
            int nseen = 0;
            bool few = true;
            for (size_t k = i; k < j && few; ++k) {
                const int64_t dk = delta(fl[k]);
                int s = 0;
                while (s < nseen && seen[s] != dk) ++s;
                if (s == nseen) {
                    if (nseen == 4) few = false;
                    else seen[nseen++] = dk;
                }
            }
            if (few && nseen > 1) {  // a stable partition by increasing offset
                std::sort(seen, seen + nseen);
                part.clear();
                for (int s = 0; s < nseen; ++s)
                    for (size_t k = i; k < j; ++k)
                        if (delta(fl[k]) == seen[s]) part.push_back(fl[k]);
                std::copy(part.begin(), part.end(), fl.begin() + (int64_t)i);
            }
            i = j;
        }
    }
    for (size_t c = 0; c < class_key.size(); ++c) {
        const int32_t kind = std::get<0>(class_key[c]);
        const std::vector<int32_t> &facs = class_facs[c];
        FGroup grp;
        grp.kind = kind;
        grp.a = 0;
        grp.b = 0;
        if (kind == TK_PAIR) {
            const int32_t na = std::get<1>(class_key[c]), nb = std::get<2>(class_key[c]);
            grp.a = na;
            grp.b = nb;
            // Tiles take 64 consecutive factors, but a tile whose factors so
            // far form one (block, variable offset) group closes early where
            // that group ends, once 48 lanes are filled: a grid's tiles then
            // each hold one run of horizontal or vertical factors, whose slot
            // variables are consecutive lanes.  Graphs whose offsets scatter
            // keep full tiles.
            auto group = [&](size_t i) {
                const int64_t e0 = d->factor_edge_off[facs[i]];
                return std::make_pair((int64_t)d->edge_var[e0] / kLanes,
                                      (int64_t)d->edge_var[e0 + 1] - d->edge_var[e0]);
            };
            for (size_t i0 = 0, len = 0; i0 < facs.size(); i0 += len) {
                len = std::min<size_t>(kLanes, facs.size() - i0);
                if (len > 48 && group(i0) == group(i0 + 47)) {
                    size_t l = 1;
                    while (l < len && group(i0 + l) == group(i0)) ++l;
                    if (l >= 48) len = l;  // one run up to lane l (else the run broke early: a full tile)
                }
                FTile ft{};
                ft.kind = TK_PAIR;
                ft.a = na;
                ft.b = nb;
                ft.nact = (int32_t)len;
                ft.m_off = (int32_t)M;
                ft.phi_off = (int32_t)P;
                ft.vb_off = (int32_t)L->fvb.size();
                add_vb_rows(2);
                for (int32_t l = 0; l < ft.nact; ++l) {
                    const int64_t f = facs[i0 + l], e0 = d->factor_edge_off[f];
                    L->edge_maddr[e0] = (int32_t)(M + l);
                    L->edge_maddr[e0 + 1] = (int32_t)(M + (int64_t)na * kLanes + l);
                    L->fvb[ft.vb_off + l] = vaddr[d->edge_var[e0]];
                    L->fvb[ft.vb_off + kLanes + l] = vaddr[d->edge_var[e0 + 1]];
                    L->fvar[ft.vb_off + l] = d->edge_var[e0];
                    L->fvar[ft.vb_off + kLanes + l] = d->edge_var[e0 + 1];
                    L->fac_phi[f] = (int32_t)(P + l);
                    tile_fac[L->ftile.size() * kLanes + l] = (int32_t)f;
                }
                M += (int64_t)kLanes * (na + nb);
                P += (int64_t)kLanes * na * nb;
                if ((rc = check(M, "message array")) || (rc = check(P, "potential array"))) return rc;
                grp.tiles.push_back((int32_t)L->ftile.size());
                L->ftile.push_back(ft);
            }
        } else if (kind == TK_LOGL) {
            const int32_t k = std::get<1>(class_key[c]), flip = std::get<2>(class_key[c]);
            for (size_t i0 = 0; i0 < facs.size(); i0 += kLanes) {
                FTile ft{};
                ft.kind = TK_LOGL;
                ft.a = k;
                ft.b = flip;
                ft.nact = (int32_t)std::min<size_t>(kLanes, facs.size() - i0);
                ft.m_off = (int32_t)M;
                ft.vb_off = (int32_t)L->fvb.size();
                add_vb_rows(k);
                for (int32_t l = 0; l < ft.nact; ++l) {
                    const int64_t f = facs[i0 + l], e0 = d->factor_edge_off[f];
                    for (int32_t j = 0; j < k; ++j) {
                        L->edge_maddr[e0 + j] = (int32_t)(M + (int64_t)2 * j * kLanes + l);
                        L->fvb[ft.vb_off + j * kLanes + l] = vaddr[d->edge_var[e0 + j]];
                        L->fvar[ft.vb_off + j * kLanes + l] = d->edge_var[e0 + j];
                    }
                }
                M += (int64_t)kLanes * 2 * k;
                if ((rc = check(M, "message array"))) return rc;
                grp.tiles.push_back((int32_t)L->ftile.size());
                L->ftile.push_back(ft);
            }
        } else if (kind == TK_LOGW) {
            grp.a = std::get<1>(class_key[c]);
            for (int32_t f : facs) {
                const int64_t e0 = d->factor_edge_off[f];
                const int32_t k = (int32_t)(d->factor_edge_off[f + 1] - e0);
                const int32_t chunks = (k + kLanes - 1) / kLanes;
                FTile ft{};
                ft.kind = TK_LOGW;
                ft.a = k;
                ft.b = d->factor_kind[f] == LBP_FACTOR_AND;
                ft.nact = 1;
                ft.m_off = (int32_t)M;
                ft.vb_off = (int32_t)L->fvb.size();
                add_vb_rows(chunks);
                for (int32_t j = 0; j < k; ++j) {
                    const int32_t ch = j / kLanes, l = j % kLanes;
                    L->edge_maddr[e0 + j] = (int32_t)(M + (int64_t)ch * 2 * kLanes + l);
                    L->fvb[ft.vb_off + j] = vaddr[d->edge_var[e0 + j]];
                    L->fvar[ft.vb_off + j] = d->edge_var[e0 + j];
                }
                M += (int64_t)chunks * 2 * kLanes;
                if ((rc = check(M, "message array"))) return rc;
                grp.tiles.push_back((int32_t)L->ftile.size());
                L->ftile.push_back(ft);
            }
        } else {  // TK_GEN
            const int32_t k = std::get<1>(class_key[c]);
            const int32_t t = std::get<3>(class_key[c]);
            const std::vector<int32_t> &ns = std::get<4>(class_key[c]);
            GenClass gc{};
            gc.arity = k;
            int32_t rows = 0;
            for (int32_t j = 0; j < k; ++j) {
                gc.slot_n[j] = ns[j];
                gc.slot_row[j] = rows;
                rows += ns[j];
            }
            gc.nrows = rows;
            gc.rows_off = (int32_t)L->grows.size();
            if (t < 0) {  // dense: every joint state, last slot fastest
                int64_t ncfg = 1;
                for (int32_t j = 0; j < k; ++j) ncfg *= ns[j];
                gc.ncfg = (int32_t)ncfg;
                for (int64_t cfg = 0; cfg < ncfg; ++cfg) {
                    int64_t r = cfg;
                    std::vector<int32_t> st(k);
                    for (int32_t j = k - 1; j >= 0; --j) {
                        st[j] = (int32_t)(r % ns[j]);
                        r /= ns[j];
                    }
                    for (int32_t j = 0; j < k; ++j) L->grows.push_back((uint8_t)(gc.slot_row[j] + st[j]));
                }
            } else {
                gc.ncfg = d->cfg_table_num_cfgs[t];
                const int32_t *st = d->cfg_table_states + d->cfg_table_off[t];
                for (int64_t cfg = 0; cfg < gc.ncfg; ++cfg)
                    for (int32_t j = 0; j < k; ++j)
                        L->grows.push_back((uint8_t)(gc.slot_row[j] + st[cfg * k + j]));
            }
            const int32_t gidx = (int32_t)L->gcls.size();
            L->gcls.push_back(gc);
            // launch groups: dense three-way classes with 2..4 states in every
            // slot run in registers (code -N); the others by LDS need
            const bool tri = t < 0 && k == 3 && ns[0] == ns[1] && ns[1] == ns[2] && ns[0] >= 2 && ns[0] <= 4;
            grp.a = tri ? -ns[0] : gen_lds_code(gc.ncfg * gc.arity, gc.nrows);
            for (size_t i0 = 0; i0 < facs.size(); i0 += kLanes) {
                FTile ft{};
                ft.kind = TK_GEN;
                ft.a = gidx;
                ft.nact = (int32_t)std::min<size_t>(kLanes, facs.size() - i0);
                ft.m_off = (int32_t)M;
                ft.phi_off = (int32_t)P;
                ft.vb_off = (int32_t)L->fvb.size();
                add_vb_rows(k);
                for (int32_t l = 0; l < ft.nact; ++l) {
                    const int64_t f = facs[i0 + l], e0 = d->factor_edge_off[f];
                    for (int32_t j = 0; j < k; ++j) {
                        L->edge_maddr[e0 + j] = (int32_t)(M + (int64_t)gc.slot_row[j] * kLanes + l);
                        L->fvb[ft.vb_off + j * kLanes + l] = vaddr[d->edge_var[e0 + j]];
                        L->fvar[ft.vb_off + j * kLanes + l] = d->edge_var[e0 + j];
                    }
                    L->fac_phi[f] = (int32_t)(P + l);
                    tile_fac[L->ftile.size() * kLanes + l] = (int32_t)f;
                }
                M += (int64_t)kLanes * rows;
                P += (int64_t)kLanes * gc.ncfg;
                if ((rc = check(M, "message array")) || (rc = check(P, "potential array"))) return rc;
                grp.tiles.push_back((int32_t)L->ftile.size());
                L->ftile.push_back(ft);
            }
        }
        // logical tiles of at most 4 chunks share one launch group; wider ones
        // another; pairwise and generic classes are one group each
        if (kind == TK_LOGL || (kind == TK_LOGW && grp.a <= 4)) {
            grp.kind = TK_LOGL;
            grp.a = 0;
        } else if (kind == TK_LOGW) {
            grp.a = 0;
        }
        bool merged = false;
        if (grp.kind == TK_LOGL || grp.kind == TK_LOGW)
            for (FGroup &g : L->fgroups)
                if (g.kind == grp.kind) {
                    g.tiles.insert(g.tiles.end(), grp.tiles.begin(), grp.tiles.end());
                    merged = true;
                }
        if (!merged) L->fgroups.push_back(grp);
    }
    // In the shared logical launch the wavefront-per-factor tiles (long
    // chains: gathers, then wavefront scans) start first, the widest first,
    // before the lane tiles fill the machine; launch order changes no
    // element's arithmetic.
    for (FGroup &g : L->fgroups) {
        if (g.kind != TK_LOGL) continue;
        std::stable_sort(g.tiles.begin(), g.tiles.end(), [&](int32_t x, int32_t y) {
            const FTile &a = L->ftile[x], &b = L->ftile[y];
            const int32_t ka = a.kind == TK_LOGW ? a.a : 0, kb = b.kind == TK_LOGW ? b.a : 0;
            return ka > kb;
        });
    }
    L->zero_addr = (int32_t)M;
    M += (int64_t)kLanes * kLowStatesMax;
    L->M = M;
    L->P = P > 0 ? P : kLanes;

    // ------------------------------------------------ variable edge-address rows
    L->vns.assign(nvt * kLanes, 0);
    L->vedge.reserve((size_t)E + 16 * kLanes);  // rows of low-degree lanes: about one entry per edge
    L->hedge.reserve((size_t)E / 4 + kLanes);
    std::map<int32_t, size_t> vgroup_of;
    auto degree = [&](int64_t v) { return adj_off[v + 1] - adj_off[v]; };
    auto edge_addr = [&](int64_t v, int64_t k) { return L->edge_maddr[adj[adj_off[v] + k]]; };
    // Column group of w variables from v (inside [v, vend) of one var tile),
    // all on the block path with v's state count.  Its edge rows pair up
    // messages that sit side by side: variable v + l's edge at message
    // address a goes to the row keyed a - l, rows in increasing key order,
    // -1 where a variable has no edge of that key.  A lane's edges then come
    // in increasing address order.  Taken when edges fill at least 3/4 of the
    // rows' entries.  The rows are a w-way merge of the variables' addresses,
    // sorted once per variable; the merge stops as soon as the rows can no
    // longer be 3/4 full.
    std::vector<int32_t> saddr;  // block-path variables' edge addresses, ascending, at adj_off[v]
    std::vector<char> sorted_v;
    auto sorted_addr = [&](int64_t u) {
        if (saddr.empty()) {
            saddr.assign(E, 0);
            sorted_v.assign(V, 0);
        }
        if (!sorted_v[u]) {
            for (int64_t k = 0; k < degree(u); ++k) saddr[adj_off[u] + k] = edge_addr(u, k);
            if (!std::is_sorted(saddr.begin() + adj_off[u], saddr.begin() + adj_off[u + 1]))
                std::sort(saddr.begin() + adj_off[u], saddr.begin() + adj_off[u + 1]);
            sorted_v[u] = 1;
        }
        return saddr.data() + adj_off[u];
    };
    auto column_rows = [&](int64_t v, int64_t w, int64_t vend, std::vector<int32_t> *rows) {
        if (v + w > vend) return false;
        int64_t edges = 0;
        for (int64_t u = v; u < v + w; ++u) {
            if (degree(u) <= kMidDegMax || L->vn[u] != L->vn[v]) return false;
            edges += degree(u);
        }
        const int32_t *a[kColLanesMax];
        int64_t pos[kColLanesMax], len[kColLanesMax];
        for (int64_t l = 0; l < w; ++l) {
            a[l] = sorted_addr(v + l);
            pos[l] = 0;
            len[l] = degree(v + l);
        }
        // the rows are at least the distinct keys of the first two lanes:
        // a cheap test that rejects most variables that form no group
        {
            const int64_t cap = 4 * edges / (3 * w);  // the most rows a taken group has
            int64_t i = 0, j = 0, keys = 0;
            while ((i < len[0] || j < len[1]) && keys <= cap) {
                const int64_t k0 = i < len[0] ? (int64_t)a[0][i] : INT64_MAX;
                const int64_t k1 = j < len[1] ? (int64_t)a[1][j] - 1 : INT64_MAX;
                i += k0 <= k1;
                j += k1 <= k0;
                ++keys;
            }
            if (keys > cap) return false;
        }
        rows->clear();
        for (int64_t left = edges; left > 0;) {
            if (4 * edges < 3 * (int64_t)(rows->size() + w)) return false;  // one more row: below 3/4 full
            int64_t key = INT64_MAX;
            for (int64_t l = 0; l < w; ++l)
                if (pos[l] < len[l]) key = std::min<int64_t>(key, (int64_t)a[l][pos[l]] - l);
            for (int64_t l = 0; l < w; ++l) {
                const bool take = pos[l] < len[l] && (int64_t)a[l][pos[l]] - l == key;
                rows->push_back(take ? a[l][pos[l]++] : -1);
                left -= take;
            }
        }
        return true;
    };
    std::vector<int32_t> col_rows;
    for (int64_t t = 0; t < nvt; ++t) {
        int32_t kmax = 0, nlow = 0;
        const int64_t v0 = t * kLanes, v1 = std::min<int64_t>(V, v0 + kLanes);
        for (int64_t v = v0; v < v1; ++v) {
            int64_t deg = degree(v);
            const bool low = deg <= kLowDegMax && L->vn[v] <= kLowStatesMax;
            if (low) {
                kmax = std::max<int32_t>(kmax, (int32_t)deg);
                nlow = std::max<int32_t>(nlow, L->vn[v]);
                L->vns[v] = L->vn[v];
                continue;
            }
            // the widest group that leaves each of its 256 threads at most
            // about 16 edges, between 4 and 16 variables
            int64_t w = 0;
            if (deg > kMidDegMax) {
                int64_t w0 = kColLanesMax;
                while (w0 > kColLanesMin && w0 * deg > 256 * 16) w0 /= 2;
                for (int64_t c = w0; c >= kColLanesMin && !w; c /= 2)
                    if (column_rows(v, c, v1, &col_rows)) w = c;
            }
            HVar h{};
            h.b_addr = vaddr[v];
            h.n = (int16_t)L->vn[v];
            h.lanes = (int16_t)std::max<int64_t>(w, 1);
            h.e_begin = (int32_t)L->hedge.size();
            if (w) {
                L->hedge.insert(L->hedge.end(), col_rows.begin(), col_rows.end());
                v += w - 1;
            } else {
                for (int64_t i = adj_off[v]; i < adj_off[v + 1]; ++i) L->hedge.push_back(L->edge_maddr[adj[i]]);
            }
            h.e_end = (int32_t)L->hedge.size();
            (w ? L->cols : deg <= kMidDegMax ? L->mids : L->highs).push_back((int32_t)L->hvar.size());
            L->hvar.push_back(h);
        }
        VTile &vt = L->vtile[t];
        vt.kmax = kmax;
        vt.e_off = (int32_t)L->vedge.size();
        L->vedge.resize(L->vedge.size() + (size_t)kmax * kLanes);
        for (int32_t k = 0; k < kmax; ++k)
            for (int32_t l = 0; l < kLanes; ++l) {
                const int64_t v = v0 + l;
                int32_t a = L->zero_addr + l;
                if (v < v1 && L->vns[v] > 0 && k < adj_off[v + 1] - adj_off[v])
                    a = L->edge_maddr[adj[adj_off[v] + k]];
                L->vedge[vt.e_off + (size_t)k * kLanes + l] = a;
            }
        if (nlow > 0) {
            int32_t b = state_bucket(nlow);
            auto it = vgroup_of.find(b);
            if (it == vgroup_of.end()) {
                vgroup_of[b] = L->vgroups.size();
                L->vgroups.push_back(VGroup{b, {}});
                it = vgroup_of.find(b);
            }
            L->vgroups[it->second].tiles.push_back((int32_t)t);
        }
    }
    if (L->vedge.size() >= (size_t)INT32_MAX || L->hedge.size() >= (size_t)INT32_MAX ||
        L->fvb.size() >= (size_t)INT32_MAX)
        return bad(err, "index tables exceed 2^31 entries", LBP_E_UNSUPPORTED);

    // pairwise slots whose lanes hold consecutive variables (grids: nearly
    // every tile) are described by their first variable, so the fused kernel
    // reads one value per slot instead of one per lane
    L->faff.assign(2 * L->ftile.size(), -1);
    for (size_t t = 0; t < L->ftile.size(); ++t) {
        const FTile &ft = L->ftile[t];
        if (ft.kind != TK_PAIR || ft.nact < 1) continue;
        for (int32_t r = 0; r < 2; ++r) {
            const int32_t *fv = L->fvar.data() + ft.vb_off + (size_t)r * kLanes;
            bool affine = true;
            for (int32_t l = 1; l < ft.nact && affine; ++l) affine = fv[l] == fv[0] + l;
            if (affine) L->faff[2 * t + r] = fv[0];
        }
    }
    L->fusable = L->hvar.empty() && !L->fgroups.empty();
    for (const FGroup &fg : L->fgroups)
        if (fg.kind != TK_PAIR || fg.a != fg.b) L->fusable = false;

    // -------------------------------------------------------------- values
    if (!fill) {
        L->tile_fac.swap(tile_fac);  // fill_panels needs it later
        return LBP_OK;
    }
    L->theta_panel.resize(L->VB);
    L->phi_panel.resize(L->P);
    L->tile_fac.swap(tile_fac);
    rc = fill_panels(d_in, *L, L->theta_panel.data(), L->phi_panel.data(), err);
    std::vector<int32_t>().swap(L->tile_fac);
    return rc;
}

int fill_panels(const lbp_graph_desc *d, const HostLayout &L, float *theta, float *phi, std::string *err) {
    // Panels are written front to back, every element once (padding zero).
    const int64_t V = L.V;
    const int64_t nvt = (int64_t)L.vtile.size();
    int64_t filled = 0;
    for (int64_t t = 0; t < nvt; ++t) {
        const VTile &vt = L.vtile[t];
        float *row = theta + vt.b_off;
        for (int32_t s = 0; s < vt.n; ++s, row += kLanes)
            for (int32_t l = 0; l < kLanes; ++l) {
                const int64_t v = t * kLanes + l;
                row[l] = (d->evidence && v < V && s < L.vn[v]) ? d->evidence[L.vs_off[v] + s] : 0.0f;
            }
        filled = std::max<int64_t>(filled, vt.b_off + (int64_t)vt.n * kLanes);
    }
    std::fill(theta + filled, theta + L.VB, 0.0f);  // the spare zero panel
    // each tile's panel is the transpose of its factors' tables: blocks of 16
    // lanes, so every configuration row is written 64 bytes at a time; the
    // values are checked for NaN and infinity on the way.  Where all 16 lanes
    // hold a factor, 4 configurations of each are read at once (16-byte
    // loads) and written out as 4 rows.
    uint32_t nonfinite = 0;
    auto flag = [](const float *x) {
        uint32_t u[16], acc = 0;
        std::memcpy(u, x, sizeof u);
        for (int32_t l = 0; l < 16; ++l) acc |= (uint32_t)((u[l] & 0x7f800000u) == 0x7f800000u);
        return acc;
    };
    for (size_t t = 0; t < L.ftile.size(); ++t) {
        const FTile &ft = L.ftile[t];
        if (ft.kind != TK_PAIR && ft.kind != TK_GEN) continue;
        const int32_t ncfg = ft.kind == TK_PAIR ? ft.a * ft.b : L.gcls[ft.a].ncfg;
        const int32_t *lf = L.tile_fac.data() + t * kLanes;
        float *panel = phi + ft.phi_off;
        for (int32_t l0 = 0; l0 < kLanes; l0 += 16) {
            const float *src[16];
            bool full = true;
            for (int32_t l = 0; l < 16; ++l) {
                src[l] = lf[l0 + l] >= 0 ? d->log_potentials + L.lp_off[lf[l0 + l]] : nullptr;
                full = full && src[l];
            }
            int32_t c = 0;
            if (full)
                for (; c + 4 <= ncfg; c += 4) {
                    alignas(16) float in[16][4];
                    for (int32_t l = 0; l < 16; ++l) std::memcpy(in[l], src[l] + c, sizeof in[l]);
                    for (int32_t j = 0; j < 4; ++j) {
                        alignas(16) float row[16];
                        for (int32_t l = 0; l < 16; ++l) row[l] = in[l][j];
                        nonfinite |= flag(row);
                        std::memcpy(panel + (int64_t)(c + j) * kLanes + l0, row, sizeof row);
                    }
                }
            for (; c < ncfg; ++c) {
                alignas(16) float row[16];
                for (int32_t l = 0; l < 16; ++l) row[l] = src[l] ? src[l][c] : 0.0f;
                nonfinite |= flag(row);
                std::memcpy(panel + (int64_t)c * kLanes + l0, row, sizeof row);
            }
        }
    }
    if (nonfinite) {
        const int64_t i = first_nonfinite(d->log_potentials, L.Tn);
        return bad(err, at("log_potentials", i) + " is not finite");
    }
    return LBP_OK;
}

int check_potentials_finite(const lbp_graph_desc *d, int64_t Tn, std::string *err) {
    const int64_t i = Tn > 0 ? first_nonfinite(d->log_potentials, Tn) : -1;
    return i >= 0 ? nonfinite_potential(i, err) : LBP_OK;
}

int nonfinite_potential(int64_t i, std::string *err) { return bad(err, at("log_potentials", i) + " is not finite"); }

int64_t copy_check_finite(float *dst, const float *src, int64_t n) {
    constexpr int64_t B = 4096;
    int64_t first = -1;
    for (int64_t b = 0; b < n; b += B) {
        const int64_t e = std::min(n, b + B);
        uint32_t hit = 0;
        for (int64_t i = b; i < e; ++i) {
            uint32_t u;
            std::memcpy(&u, src + i, sizeof u);
            std::memcpy(dst + i, &u, sizeof u);
            hit |= (uint32_t)((u & 0x7f800000u) == 0x7f800000u);
        }
        if (hit && first < 0)
            for (int64_t i = b; i < e; ++i)
                if (!std::isfinite(dst[i])) {
                    first = i;
                    break;
                }
    }
    return first;
}

// Replays the address arithmetic of every kernel over the compiled layout and
// checks each access against its array's size.  Host only.
int check_layout(const HostLayout &L, std::string *err) {
    const int64_t M = L.M, VB = L.VB, P = L.P;
    auto oob = [&](const std::string &what) { return bad(err, "layout check: " + what); };
    auto in = [](int64_t a, int64_t n) { return a >= 0 && a < n; };
    // rows a, a + 64, ..., a + 64 (k - 1) all inside [0, n): the ends suffice
    auto rows_in = [](int64_t a, int64_t k, int64_t n) { return k <= 0 || (a >= 0 && a + (k - 1) * kLanes < n); };
    // variable phase, low-degree lanes
    for (const VGroup &vg : L.vgroups)
        for (int32_t t : vg.tiles) {
            if (!in(t, (int64_t)L.vtile.size())) return oob("var tile index");
            const VTile &vt = L.vtile[t];
            for (int32_t l = 0; l < kLanes; ++l) {
                const int32_t n = L.vns[(size_t)t * kLanes + l];
                if (n > vg.bucket || n > vt.n) return oob("lane states exceed bucket/panel");
                if (!rows_in(vt.b_off + l, n, VB)) return oob("belief-low B/theta");
                for (int32_t k = 0; k < vt.kmax; ++k) {
                    const int64_t ei = vt.e_off + (int64_t)k * kLanes + l;
                    if (!in(ei, (int64_t)L.vedge.size())) return oob("vedge index");
                    if (!rows_in(L.vedge[ei], n, M)) return oob("belief-low message");
                }
            }
        }
    // variable phase, wavefront- and block-per-variable paths
    for (int32_t i : L.mids)
        if (!in(i, (int64_t)L.hvar.size()) || L.hvar[i].e_end - L.hvar[i].e_begin > kMidDegMax ||
            L.hvar[i].lanes != 1)
            return oob("wavefront-per-variable entry");
    for (int32_t i : L.highs)
        if (!in(i, (int64_t)L.hvar.size()) || L.hvar[i].lanes != 1) return oob("block-per-variable entry");
    std::vector<char> block_path(L.hvar.size(), 0);
    for (int32_t i : L.cols) {
        if (!in(i, (int64_t)L.hvar.size()) || L.hvar[i].lanes == 1) return oob("column group entry");
        block_path[i] = 1;
    }
    if (L.mids.size() + L.highs.size() + L.cols.size() != L.hvar.size()) return oob("variable path lists");
    for (size_t i = 0; i < L.hvar.size(); ++i) {
        const HVar &h = L.hvar[i];
        if (h.e_begin < 0 || h.e_end < h.e_begin || h.e_end > (int64_t)L.hedge.size()) return oob("hedge range");
        // a column group: a power of two of variables in one panel row
        // (b_addr .. b_addr + lanes - 1 share the row), on the block path,
        // whole edge rows; -1 entries are skipped
        const int32_t w = h.lanes;
        const bool col = w != 1;
        if (col && (w < kColLanesMin || w > kColLanesMax || (w & (w - 1)) || !block_path[i] ||
                    (h.e_end - h.e_begin) % w != 0 || h.b_addr % kLanes + w > kLanes))
            return oob("column group");
        for (int32_t l = 0; l < w; ++l)
            if (!rows_in(h.b_addr + l, h.n, VB)) return oob("belief-high B/theta");
        for (int32_t k = h.e_begin; k < h.e_end; ++k)
            if (!(col && L.hedge[k] == -1) && !rows_in(L.hedge[k], h.n, M)) return oob("belief-high message");
    }
    // factor phase
    auto vb_rows = [&](const FTile &ft, int32_t rows, const int32_t *row_n) -> bool {
        for (int32_t r = 0; r < rows; ++r)
            for (int32_t l = 0; l < kLanes; ++l) {
                const int64_t i = ft.vb_off + (int64_t)r * kLanes + l;
                if (!in(i, (int64_t)L.fvb.size()) || !rows_in(L.fvb[i], row_n[r], VB)) return false;
            }
        return true;
    };
    for (const FGroup &fg : L.fgroups)
        for (int32_t t : fg.tiles) {
            if (!in(t, (int64_t)L.ftile.size())) return oob("factor tile index");
            const FTile &ft = L.ftile[t];
            const bool kind_ok = ft.kind == fg.kind ||
                                 (fg.kind == TK_LOGL && ft.kind == TK_LOGW && ft.a <= 4 * kLanes);
            if (!kind_ok) return oob("tile kind differs from its launch group");
            if (ft.kind == TK_PAIR) {
                const int32_t ns[2] = {ft.a, ft.b};
                if (ft.a > kPairStatesMax || ft.b > kPairStatesMax) return oob("pair states");
                if (fg.a != ft.a || fg.b != ft.b) return oob("pair group shape");
                if (!vb_rows(ft, 2, ns)) return oob("pair belief rows");
                if (!in(ft.m_off + (int64_t)(ft.a + ft.b) * kLanes - 1, M)) return oob("pair messages");
                if (!in(ft.phi_off + (int64_t)ft.a * ft.b * kLanes - 1, P)) return oob("pair potentials");
            } else if (ft.kind == TK_LOGL) {
                if (ft.a < 2 || ft.a > kLogLaneArityMax) return oob("lane logical arity");
                const int32_t ns[kLogLaneArityMax] = {2, 2, 2, 2, 2, 2, 2, 2};
                if (!vb_rows(ft, ft.a, ns)) return oob("lane logical belief rows");
                if (!in(ft.m_off + (int64_t)2 * ft.a * kLanes - 1, M)) return oob("lane logical messages");
            } else if (ft.kind == TK_LOGW) {
                const int32_t ch = (ft.a + kLanes - 1) / kLanes;
                if (ft.a < 2 || ft.a > kLogWaveArityMax || (fg.kind == TK_LOGL && ch > 4))
                    return oob("wave logical arity/bucket");
                for (int32_t j = 0; j < ft.a; ++j) {
                    const int64_t i = ft.vb_off + j;
                    if (!in(i, (int64_t)L.fvb.size()) || !in(L.fvb[i] + kLanes, VB)) return oob("wave logical beliefs");
                }
                if (!in(ft.m_off + (int64_t)ch * 2 * kLanes - 1, M)) return oob("wave logical messages");
            } else if (ft.kind == TK_GEN) {
                if (!in(ft.a, (int64_t)L.gcls.size())) return oob("generic class index");
                const GenClass &gc = L.gcls[ft.a];
                if (gc.arity > kGenArityMax || gc.ncfg > kGenCfgMax || gc.nrows > kGenRowsMax) return oob("generic limits");
                if (fg.a < 0) {  // the register kernel: a dense three-way class with -a states per slot
                    const int N = -fg.a;
                    if (gc.arity != 3 || gc.ncfg != N * N * N || gc.nrows != 3 * N) return oob("three-way class");
                    for (int32_t j = 0; j < 3; ++j)
                        if (gc.slot_n[j] != N || gc.slot_row[j] != j * N) return oob("three-way slots");
                    for (int32_t c = 0; c < gc.ncfg; ++c)  // dense order, last slot fastest
                        for (int32_t j = 0; j < 3; ++j) {
                            const int32_t st = j == 0 ? c / (N * N) : j == 1 ? (c / N) % N : c % N;
                            if (L.grows[gc.rows_off + (int64_t)c * 3 + j] != j * N + st) return oob("three-way table");
                        }
                } else if (fg.a != 0) {  // the dynamic-LDS kernel: the class must fit the group's LDS
                    int rb, nr;
                    gen_lds_decode(fg.a, &rb, &nr);
                    if ((int64_t)gc.ncfg * gc.arity > rb || gc.nrows > nr) return oob("generic class exceeds its LDS");
                }
                if (gc.rows_off + (int64_t)gc.ncfg * gc.arity > (int64_t)L.grows.size()) return oob("generic rows");
                for (int64_t i = 0; i < (int64_t)gc.ncfg * gc.arity; ++i)
                    if (L.grows[gc.rows_off + i] >= gc.nrows) return oob("generic row entry");
                if (!vb_rows(ft, gc.arity, gc.slot_n)) return oob("generic belief rows");
                if (!in(ft.m_off + (int64_t)gc.nrows * kLanes - 1, M)) return oob("generic messages");
                if (!in(ft.phi_off + (int64_t)gc.ncfg * kLanes - 1, P)) return oob("generic potentials");
            } else {
                return oob("unknown tile kind");
            }
        }
    // read-out and flat-order exchange
    if (!L.vext.empty()) {
        if ((int64_t)L.vext.size() != L.V) return oob("variable order size");
        for (int64_t v = 0; v < L.V; ++v)
            if (!in(L.vext[v], L.V)) return oob("variable order entry");
    }
    for (int64_t v = 0; v < L.V; ++v) {
        const VTile &vt = L.vtile[v / kLanes];
        if (L.vn[v] > vt.n) return oob("read-out panel rows");
        if (!in(vt.b_off + v % kLanes + (int64_t)(L.vn[v] - 1) * kLanes, VB)) return oob("read-out beliefs");
    }
    for (int64_t e = 0; e < L.E; ++e) {
        const int64_t n = L.es_off[e + 1] - L.es_off[e];
        if (!in(L.edge_maddr[e] + (n - 1) * kLanes, M)) return oob("edge message address");
    }
    for (int64_t f = 0; f < L.F; ++f)
        if (L.fac_phi[f] >= 0 && !in(L.fac_phi[f] + (L.lp_off[f + 1] - L.lp_off[f] - 1) * kLanes, P))
            return oob("factor potential address");
    if (!in(L.zero_addr + (int64_t)kLowStatesMax * kLanes - 1, M)) return oob("zero panel");
    if (L.fvar.size() != L.fvb.size()) return oob("fvar size");
    if (L.faff.size() != 2 * L.ftile.size()) return oob("slot base size");
    for (size_t t = 0; t < L.ftile.size(); ++t)
        for (int32_t r = 0; r < 2; ++r) {
            const int32_t v0 = L.faff[2 * t + r];
            if (v0 < 0) continue;
            const FTile &ft = L.ftile[t];
            if (ft.kind != TK_PAIR) return oob("slot base of a non-pairwise tile");
            for (int32_t l = 0; l < ft.nact; ++l)
                if (L.fvar[ft.vb_off + (int64_t)r * kLanes + l] != v0 + l) return oob("slot base");
        }
    if (L.fusable) {
        // the fused pairwise kernel recomputes each slot variable's belief from
        // its edge rows: the variable's tile, lane states and edge addresses
        // (checked once per variable, then per slot that the variable and its
        // state count are the tile's)
        std::vector<char> rows_ok(L.V);
        for (int64_t v = 0; v < L.V; ++v) {
            const VTile &vt = L.vtile[v / kLanes];
            const int32_t n = L.vns[v];
            bool ok = in(vt.b_off + v % kLanes + (int64_t)(n - 1) * kLanes, VB);
            for (int32_t k = 0; ok && k < vt.kmax; ++k) {
                const int64_t ei = vt.e_off + (int64_t)k * kLanes + v % kLanes;
                ok = in(ei, (int64_t)L.vedge.size()) && in(L.vedge[ei] + (int64_t)(n - 1) * kLanes, M);
            }
            rows_ok[v] = ok;
        }
        for (const FGroup &fg : L.fgroups)
            for (int32_t t : fg.tiles) {
                const FTile &ft = L.ftile[t];
                for (int32_t r = 0; r < 2; ++r)
                    for (int32_t l = 0; l < ft.nact; ++l) {
                        const int32_t v = L.fvar[ft.vb_off + (int64_t)r * kLanes + l];
                        if (!in(v, L.V)) return oob("fused slot variable");
                        if (L.vns[v] != (r == 0 ? ft.a : ft.b)) return oob("fused slot states");
                        if (!rows_ok[v]) return oob("fused edge rows or evidence");
                    }
            }
    }
    return LBP_OK;
}

}  // namespace lbp
