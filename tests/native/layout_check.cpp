// Host-only test of the layout check (check_layout): a compiled layout that
// mixes every tile kind passes, and each single corruption of an address,
// offset or table that a kernel would follow out of its array is rejected
// with the matching message.  Built and run by tests/test_layout_check.py.
#include <cstdio>
#include <functional>
#include <utility>
#include <string>
#include <vector>

#include "../../paper_2202_04110_amd/csrc/compile.h"
#include "desc_builder.h"

using namespace lbp;
using lbp_test::Builder;

namespace {

int failures = 0;

void expect(bool ok, const std::string &what) {
    if (!ok) {
        std::printf("FAIL: %s\n", what.c_str());
        ++failures;
    }
}

// Compiles `b`, checks the clean layout, then applies each corruption to a
// fresh copy and expects check_layout to reject it with `msg` in the error.
void run(const char *name, Builder &b,
         const std::vector<std::pair<std::string, std::function<void(HostLayout &)>>> &cases) {
    HostLayout L;
    std::string err;
    int rc = compile_desc(b.desc(), &L, &err);
    expect(rc == LBP_OK, std::string(name) + ": compile: " + err);
    if (rc != LBP_OK) return;
    rc = check_layout(L, &err);
    expect(rc == LBP_OK, std::string(name) + ": clean layout rejected: " + err);
    for (const auto &c : cases) {
        HostLayout bad = L;
        c.second(bad);
        std::string e;
        const int r = check_layout(bad, &e);
        expect(r != LBP_OK && e.find(c.first) != std::string::npos,
               std::string(name) + ": corruption '" + c.first + "' gave rc " + std::to_string(r) + " '" + e + "'");
    }
    std::printf("%s: %zu corruptions rejected (M %lld, VB %lld, P %lld, fusable %d)\n", name, cases.size(),
                (long long)L.M, (long long)L.VB, (long long)L.P, (int)L.fusable);
}

}  // namespace

int main() {
    // a 9 x 9 grid of 3-state variables: lane-path variables, dense pairwise
    // tiles, fused iterations possible
    Builder g;
    const int Lg = 9;
    for (int i = 0; i < Lg * Lg; ++i) g.var(3);
    const int t2 = g.table(2);
    for (int r = 0; r < Lg; ++r)
        for (int c = 0; c + 1 < Lg; ++c) g.enumf({r * Lg + c, r * Lg + c + 1}, t2);
    for (int r = 0; r + 1 < Lg; ++r)
        for (int c = 0; c < Lg; ++c) g.enumf({r * Lg + c, (r + 1) * Lg + c}, t2);
    run("grid", g,
        {{"belief-low message", [](HostLayout &L) { L.vedge[3] = (int32_t)L.M; }},
         {"belief-low message", [](HostLayout &L) { L.vedge[0] = -5; }},
         {"vedge index", [](HostLayout &L) { L.vtile[0].e_off = (int32_t)L.vedge.size(); }},
         {"belief-low B/theta", [](HostLayout &L) { L.vtile[1].b_off = (int32_t)L.VB - 1; }},
         {"pair belief rows", [](HostLayout &L) { L.fvb[5] = (int32_t)L.VB - 64; }},
         {"pair messages", [](HostLayout &L) { L.ftile[0].m_off = (int32_t)L.M - 64; }},
         {"pair potentials", [](HostLayout &L) { L.ftile[0].phi_off = (int32_t)L.P - 64; }},
         {"edge message address", [](HostLayout &L) { L.edge_maddr[7] = (int32_t)L.M - 1; }},
         {"factor potential address", [](HostLayout &L) { L.fac_phi[2] = (int32_t)L.P; }},
         {"fused slot variable", [](HostLayout &L) { L.fvar[1] = (int32_t)L.V; }},
         {"fused slot states", [](HostLayout &L) { L.vns[L.fvar[0]] = 2; }},
         {"zero panel", [](HostLayout &L) { L.zero_addr = (int32_t)L.M; }},
         {"slot base", [](HostLayout &L) {
              for (int32_t &v0 : L.faff)
                  if (v0 >= 0) {
                      v0 += 1;
                      break;
                  }
          }},
         {"slot base size", [](HostLayout &L) { L.faff.pop_back(); }}});

    // a hub joined to 40 and to 300 binary leaves (wavefront- and
    // block-per-variable paths), an OR over 150 parents (wavefront logical
    // tile), small ANDs (lane logical tiles) and dense three-way factors
    // (generic class)
    Builder h;
    const int hub = h.var(2), hub2 = h.var(4);
    const int tp = h.table(2), t3 = h.table(3);
    std::vector<int> leaves;
    for (int i = 0; i < 300; ++i) leaves.push_back(h.var(2));
    for (int i = 0; i < 300; ++i) h.enumf({hub, leaves[i]}, tp);
    for (int i = 0; i < 40; ++i) h.enumf({leaves[i], hub2}, tp);
    std::vector<int> orv(leaves.begin() + 40, leaves.begin() + 190);
    orv.push_back(h.var(2));
    h.logical(orv, LBP_FACTOR_OR);
    for (int i = 200; i + 2 < 230; i += 3) h.logical({leaves[i], leaves[i + 1], leaves[i + 2]}, LBP_FACTOR_AND);
    const int a3 = h.var(3), b3 = h.var(3), c3 = h.var(3);
    h.enumf({a3, b3, c3}, t3);
    h.enumf({leaves[250], a3, c3}, t3);
    run("hub", h,
        {{"belief-high message", [](HostLayout &L) { L.hedge[L.hvar[L.highs[0]].e_begin] = (int32_t)L.M - 1; }},
         {"belief-high B/theta", [](HostLayout &L) { L.hvar[L.highs[0]].b_addr = (int32_t)L.VB - 1; }},
         {"hedge range", [](HostLayout &L) { L.hvar[0].e_end = (int32_t)L.hedge.size() + 1; }},
         {"wavefront-per-variable entry", [](HostLayout &L) { L.mids[0] = (int32_t)L.hvar.size(); }},
         {"wave logical", [](HostLayout &L) {
              for (FTile &t : L.ftile)
                  if (t.kind == TK_LOGW) t.m_off = (int32_t)L.M - 64;
          }},
         {"lane logical", [](HostLayout &L) {
              for (FTile &t : L.ftile)
                  if (t.kind == TK_LOGL) t.m_off = (int32_t)L.M - 64;
          }},
         {"generic", [](HostLayout &L) {
              for (FTile &t : L.ftile)
                  if (t.kind == TK_GEN) t.phi_off = (int32_t)L.P - 1;
          }},
         {"three-way table", [](HostLayout &L) { L.grows[L.gcls[0].rows_off] = 200; }},
         {"read-out", [](HostLayout &L) { L.vn[0] = 9; }}});

    // a dense bipartite layer, 70 visible x 80 hidden binary units (every
    // unit on the block path): the hidden units' k-th edges sit side by side,
    // so they form column groups of 16, 8 and 4 units; the visible units'
    // edges run along their own rows and stay single
    Builder rb;
    const int nvis = 70, nhid = 80;
    for (int i = 0; i < nvis + nhid; ++i) rb.var(2);
    const int tr = rb.table(2);
    for (int i = 0; i < nvis; ++i)
        for (int j = 0; j < nhid; ++j) rb.enumf({i, nvis + j}, tr);
    {
        HostLayout L;
        std::string err;
        expect(compile_desc(rb.desc(), &L, &err) == LBP_OK, "bipartite: compile: " + err);
        std::vector<int> widths;
        int singles = 0;
        for (const HVar &h : L.hvar) {
            if (h.lanes > 1) widths.push_back(h.lanes);
            else ++singles;
        }
        // Every factor joins two block-path units, so the layer is ordered by
        // the 16-unit block of the hidden unit, then the visible unit: a tile
        // holds 4 visible x 16 hidden units, and hidden unit u's edge sits in
        // the lane after unit u - 1's wherever both fall in one block (units
        // 64..79, 80..95, ...).  A group never spans a block boundary (its
        // rows would be half empty) or a var tile ([64, 128), [128, 192)):
        // groups at 70 (8), 80, 96, 112, 128 (16 each) and 144 (4); units
        // 78, 79, 148 and 149 stay single, as do the 70 visible units.
        const std::vector<int> want{8, 16, 16, 16, 16, 4};
        expect(widths == want, "bipartite: column group widths");
        expect(singles == nvis + 4, "bipartite: single block-path units");
    }
    run("bipartite", rb,
        {{"column group", [](HostLayout &L) {
              for (HVar &h : L.hvar)
                  if (h.lanes > 1) {
                      h.lanes = 3;
                      break;
                  }
          }},
         {"column group", [](HostLayout &L) {
              for (HVar &h : L.hvar)
                  if (h.lanes > 1) {
                      h.b_addr += kLanes - h.lanes + 1;  // the group would leave its panel row
                      break;
                  }
          }},
         {"column group", [](HostLayout &L) {
              for (HVar &h : L.hvar)
                  if (h.lanes > 1) {
                      h.e_end -= 1;  // a partial edge row
                      break;
                  }
          }},
         {"belief-high message", [](HostLayout &L) {
              for (HVar &h : L.hvar)
                  if (h.lanes == 1) {
                      L.hedge[h.e_begin] = -1;  // skipped only inside column groups
                      break;
                  }
          }},
         {"belief-high message", [](HostLayout &L) {
              for (HVar &h : L.hvar)
                  if (h.lanes > 1) {
                      L.hedge[h.e_end - 1] = (int32_t)L.M;
                      break;
                  }
          }},
         {"block-per-variable entry", [](HostLayout &L) { std::swap(L.cols[0], L.highs[0]); }},
         {"column group entry", [](HostLayout &L) { L.cols.push_back(L.highs.back()); }},
         {"variable path lists", [](HostLayout &L) { L.cols.pop_back(); }}});

    // a small blind deconvolution: 2 activation maps of 8 units, a 3-unit
    // template each, products AND(S, W) in activation order, 10 pixels each
    // an OR over the products that land on it.  The products (two edges
    // each) are renumbered in pixel order into the ids they held; the
    // activation and template units keep theirs.
    Builder dc;
    const int K = 2, sd = 8, tw = 3, img = 10;
    std::vector<int> W, S, prod_pix;
    for (int i = 0; i < K * tw; ++i) W.push_back(dc.var(2));
    for (int i = 0; i < K * sd; ++i) S.push_back(dc.var(2));
    std::vector<std::vector<int>> pix_par(img);
    std::vector<int> prods;
    for (int k = 0; k < K; ++k)
        for (int p = 0; p < sd; ++p)
            for (int a = 0; a < tw; ++a)
                if (p + a < img) {
                    const int sw = dc.var(2);
                    prods.push_back(sw);
                    pix_par[p + a].push_back(sw);
                    dc.logical({S[k * sd + p], W[k * tw + a], sw}, LBP_FACTOR_AND);
                }
    std::vector<int> X, pad;
    for (int i = 0; i < img; ++i) X.push_back(dc.var(2));
    // parents shared by every OR (more than two edges each: never renumbered)
    // make each OR wide enough for a wavefront tile
    for (int i = 0; i < kLogLaneArityMax; ++i) pad.push_back(dc.var(2));
    for (int i = 0; i < img; ++i) {
        std::vector<int> vs = pix_par[i];
        vs.insert(vs.end(), pad.begin(), pad.end());
        vs.push_back(X[i]);
        dc.logical(vs, LBP_FACTOR_OR);
    }
    {
        HostLayout L;
        std::string err;
        expect(compile_desc(dc.desc(), &L, &err) == LBP_OK, "deconvolution: compile: " + err);
        const int64_t V = L.V;
        expect((int64_t)L.vext.size() == V, "deconvolution: variables renumbered");
        std::vector<int> inv(V, -1);
        bool perm = (int64_t)L.vext.size() == V;
        for (int64_t i = 0; perm && i < V; ++i) {
            perm = L.vext[i] >= 0 && L.vext[i] < V && inv[L.vext[i]] < 0;
            if (perm) inv[L.vext[i]] = (int)i;
        }
        expect(perm, "deconvolution: the order is a permutation");
        if (perm) {
            for (int v : W) expect(inv[v] == v, "deconvolution: template units keep their ids");
            for (int v : S) expect(inv[v] == v, "deconvolution: activation units keep their ids");
            for (int v : X) expect(inv[v] == v, "deconvolution: pixels keep their ids");
            for (int v : pad) expect(inv[v] == v, "deconvolution: shared parents keep their ids");
            // every OR factor's product parents, in its edge order, are consecutive internal ids
            int next = prods.front();
            for (int i = 0; i < img; ++i)
                for (int v : pix_par[i]) expect(inv[v] == next++, "deconvolution: OR parents consecutive");
            // the flat offsets follow the caller's order
            for (int64_t i = 0; i < V; ++i) expect(L.vs_off[i] == 2LL * L.vext[i], "deconvolution: flat offsets");
        }
    }
    run("deconvolution", dc,
        {{"variable order entry", [](HostLayout &L) { L.vext[3] = (int32_t)L.V; }},
         {"variable order size", [](HostLayout &L) { L.vext.pop_back(); }}});

    // parents shared by two wide factors (taken by the first), a parent
    // listed twice in one factor, and parents that are children elsewhere:
    // still a permutation, and the layout checks clean
    {
        Builder e;
        std::vector<int> vs;
        for (int i = 0; i < 120; ++i) vs.push_back(e.var(2));
        std::vector<int> o1, o2, o3;
        for (int i = 0; i < 30; ++i) o1.push_back(vs[(i * 37) % 120]);
        o1.push_back(vs[119]);
        for (int i = 0; i < 20; ++i) o2.push_back(vs[(i * 37) % 120]);  // the same parents again
        o2.push_back(vs[118]);
        for (int i = 0; i < 12; ++i) o3.push_back(vs[(i * 53 + 7) % 120]);
        o3.push_back(o3[0]);  // a parent twice
        o3.push_back(vs[(5 * 37) % 120]);  // a child that is also a parent above
        e.logical(o1, LBP_FACTOR_OR);
        e.logical(o2, LBP_FACTOR_AND);
        e.logical(o3, LBP_FACTOR_OR);
        HostLayout L;
        std::string err;
        expect(compile_desc(e.desc(), &L, &err) == LBP_OK, "shared parents: compile: " + err);
        std::vector<int> seen(L.V, 0);
        bool perm = L.vext.empty() || (int64_t)L.vext.size() == L.V;
        for (int32_t x : L.vext) perm = perm && x >= 0 && x < L.V && !seen[x]++;
        expect(perm, "shared parents: the order is a permutation");
        expect(check_layout(L, &err) == LBP_OK, "shared parents: layout check: " + err);
    }

    // a graph without wide logical factors keeps the caller's order
    {
        HostLayout L;
        std::string err;
        expect(compile_desc(g.desc(), &L, &err) == LBP_OK && L.vext.empty(), "grid: caller's order kept");
    }

    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("layout check ok\n");
    return 0;
}
