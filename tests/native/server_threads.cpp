// Host-only exercise of the serving scheduler's threads (client submissions
// from several threads, preparation threads, the worker, polling and
// cancellation from the caller), built with ThreadSanitizer by
// tests/test_server_tsan.py.  No GPU: the server keeps books only.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../include/lbp.h"

namespace {

// Potts-style grid (L x L, n states) with deterministic values.
struct Grid {
    std::vector<int32_t> ns, kind, ev_var, cfg, ncfg{0}, arity{2}, states;
    std::vector<int64_t> eoff{0}, coff{0, 0}, lpoff{0};
    std::vector<float> ev, lp;
    lbp_graph_desc d{};
    Grid(int L, int n, int seed) {
        const int V = L * L;
        ns.assign(V, n);
        for (int i = 0; i < V * n; ++i) ev.push_back((float)(((i * 7 + seed) % 13) - 6) * 0.1f);
        auto add = [&](int a, int b) {
            ev_var.push_back(a);
            ev_var.push_back(b);
            kind.push_back(LBP_FACTOR_ENUM);
            cfg.push_back(0);
            eoff.push_back((int64_t)ev_var.size());
            for (int c = 0; c < n * n; ++c) lp.push_back((float)((c * 5 + a + seed) % 11) * 0.05f);
            lpoff.push_back((int64_t)lp.size());
        };
        for (int r = 0; r < L; ++r)
            for (int c = 0; c + 1 < L; ++c) add(r * L + c, r * L + c + 1);
        for (int r = 0; r + 1 < L; ++r)
            for (int c = 0; c < L; ++c) add(r * L + c, (r + 1) * L + c);
        d.num_vars = V;
        d.var_num_states = ns.data();
        d.evidence = ev.data();
        d.num_factors = (int32_t)kind.size();
        d.factor_kind = kind.data();
        d.factor_edge_off = eoff.data();
        d.edge_var = ev_var.data();
        d.factor_cfg_table = cfg.data();
        d.num_cfg_tables = 1;
        d.cfg_table_num_cfgs = ncfg.data();
        d.cfg_table_arity = arity.data();
        d.cfg_table_off = coff.data();
        d.cfg_table_states = states.data();
        d.logpot_off = lpoff.data();
        d.log_potentials = lp.data();
    }
};

}  // namespace

int main() {
    const int kClients = 4, kPerClient = 40;
    std::vector<Grid> grids;
    for (int i = 0; i < 12; ++i) grids.emplace_back(6 + (i * 5) % 20, 2 + i % 5, i);
    lbp_server *srv = nullptr;
    if (lbp_server_create_host_only(int64_t(8) << 20, 6, 3, &srv) != LBP_OK) {
        std::fprintf(stderr, "create: %s\n", lbp_last_error());
        return 2;
    }
    std::atomic<int> submitted{0}, submit_errors{0};
    std::vector<std::thread> clients;
    for (int c = 0; c < kClients; ++c)
        clients.emplace_back([&, c] {
            for (int k = 0; k < kPerClient; ++k) {
                const int i = c * kPerClient + k;
                const Grid &g = grids[i % grids.size()];
                std::vector<float> gq;
                const bool backward = i % 7 == 0;
                if (backward) gq.assign(g.ev.size(), 0.5f);
                const uint64_t id = (uint64_t)i + 1;
                const int rc = lbp_server_submit(srv, &g.d, 8 + i % 9, 0.5f, 1.0f, backward ? gq.data() : nullptr, 4,
                                                 -1.0, id);
                if (rc == LBP_OK) ++submitted;
                else ++submit_errors;
            }
        });
    // poll and cancel from this thread while the clients submit
    std::vector<lbp_completion> buf(64);
    int completed = 0, ok = 0, cancelled = 0;
    for (int round = 0; round < 2000 && (completed < kClients * kPerClient); ++round) {
        if (round % 50 == 3) lbp_server_cancel(srv, (uint64_t)round % (kClients * kPerClient) + 1);
        int32_t n = 0;
        lbp_server_poll(srv, buf.data(), (int32_t)buf.size(), &n);
        for (int j = 0; j < n; ++j) {
            ++completed;
            ok += buf[j].status == LBP_OK;
            cancelled += buf[j].status == LBP_E_STATE;
        }
        if (n == 0) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    for (std::thread &t : clients) t.join();
    lbp_server_drain(srv, 60.0);
    for (;;) {
        int32_t n = 0;
        lbp_server_poll(srv, buf.data(), (int32_t)buf.size(), &n);
        if (n == 0) break;
        for (int j = 0; j < n; ++j) {
            ++completed;
            ok += buf[j].status == LBP_OK;
            cancelled += buf[j].status == LBP_E_STATE;
        }
    }
    int64_t st[18] = {0};
    lbp_server_stats(srv, st);
    lbp_server_destroy(srv);
    // concurrent host-only validation and layout checks
    std::vector<std::thread> checkers;
    std::atomic<int> check_errors{0};
    for (int c = 0; c < 4; ++c)
        checkers.emplace_back([&, c] {
            for (int k = 0; k < 10; ++k) {
                int64_t sz[6], info[4];
                const Grid &g = grids[(c * 10 + k) % grids.size()];
                if (lbp_validate(&g.d, sz) != LBP_OK || lbp_check_layout(&g.d, info) != LBP_OK) ++check_errors;
            }
        });
    for (std::thread &t : checkers) t.join();
    std::printf("submitted %d errors %d completed %d ok %d cancelled %d rounds %lld check_errors %d\n",
                submitted.load(), submit_errors.load(), completed, ok, cancelled, (long long)st[6], check_errors.load());
    const bool good = submit_errors == 0 && completed == kClients * kPerClient &&
                      ok + cancelled == completed && check_errors == 0;
    return good ? 0 : 1;
}
