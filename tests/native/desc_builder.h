// A factor-graph description built factor by factor for the host-only
// native tests (dense tables with deterministic values).
#pragma once
#include <cstdint>
#include <vector>

#include "../../include/lbp.h"

namespace lbp_test {

struct Builder {
    std::vector<int32_t> ns, kind, evar, cfg, ncfg{0}, arity, states;
    std::vector<int64_t> eoff{0}, coff{0}, lpoff{0};
    std::vector<float> ev, lp;
    lbp_graph_desc d{};

    int var(int n) {
        ns.push_back(n);
        for (int s = 0; s < n; ++s) ev.push_back(0.1f * (float)((ns.size() * 3 + s) % 7) - 0.3f);
        return (int)ns.size() - 1;
    }
    int table(int a) {  // a dense table of arity a
        const int t = (int)arity.size();
        if (t > 0) ncfg.push_back(0);
        arity.push_back(a);
        coff.push_back(0);
        return t;
    }
    void enumf(const std::vector<int> &vs, int t) {
        int64_t c = 1;
        for (int v : vs) {
            evar.push_back(v);
            c *= ns[v];
        }
        kind.push_back(LBP_FACTOR_ENUM);
        cfg.push_back(t);
        eoff.push_back((int64_t)evar.size());
        for (int64_t i = 0; i < c; ++i) lp.push_back(0.05f * (float)((i * 5 + vs[0]) % 11));
        lpoff.push_back((int64_t)lp.size());
    }
    void logical(const std::vector<int> &vs, int k) {
        for (int v : vs) evar.push_back(v);
        kind.push_back(k);
        cfg.push_back(-1);
        eoff.push_back((int64_t)evar.size());
        lpoff.push_back((int64_t)lp.size());
    }
    const lbp_graph_desc *desc() {
        d = lbp_graph_desc{};
        d.num_vars = (int32_t)ns.size();
        d.var_num_states = ns.data();
        d.evidence = ev.data();
        d.num_factors = (int32_t)kind.size();
        d.factor_kind = kind.data();
        d.factor_edge_off = eoff.data();
        d.edge_var = evar.data();
        d.factor_cfg_table = cfg.data();
        d.num_cfg_tables = (int32_t)arity.size();
        d.cfg_table_num_cfgs = ncfg.data();
        d.cfg_table_arity = arity.data();
        d.cfg_table_off = coff.data();
        d.cfg_table_states = states.data();
        d.logpot_off = lpoff.data();
        d.log_potentials = lp.data();
        return &d;
    }
};

}  // namespace lbp_test
