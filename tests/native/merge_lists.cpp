// Host-only test of the launch lists of several graphs (add_to_lists,
// finish_lists): with merging, the square pairwise classes of 2..8 states
// become one mixed launch and the variable buckets up to 8 one launch, every
// work item kept exactly once; without it, and where a class falls outside
// those limits, the per-class launches stay.  Built against liblbp.so and
// run by tests/test_merge_lists.py.
#include <algorithm>
#include <cstdio>
#include <string>
#include <tuple>
#include <vector>

#include "../../paper_2202_04110_amd/csrc/runtime.h"
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

// a side x side grid of n-state variables with dense pairwise factors
void grid(Builder &b, int side, int n) {
    const int v0 = (int)b.ns.size();
    for (int i = 0; i < side * side; ++i) b.var(n);
    const int t = b.table(2);
    for (int r = 0; r < side; ++r)
        for (int c = 0; c + 1 < side; ++c) b.enumf({v0 + r * side + c, v0 + r * side + c + 1}, t);
    for (int r = 0; r + 1 < side; ++r)
        for (int c = 0; c < side; ++c) b.enumf({v0 + r * side + c, v0 + (r + 1) * side + c}, t);
}

GraphShape shape_of(Builder &b, HostLayout &L) {
    std::string err;
    const int rc = compile_desc(b.desc(), &L, &err);
    expect(rc == LBP_OK, "compile: " + err);
    return GraphShape{L.fgroups, L.vgroups, L.mids, L.highs, L.cols};
}

using Item = std::tuple<int32_t, int32_t, int32_t>;  // (kind tag, graph, tile)

// Every (graph, tile) of the lists, tagged by launch family (variable: -1,
// factor: its kind), sorted.
std::vector<Item> items_of(const LaunchLists &ll) {
    std::vector<Item> v;
    for (const auto &l : ll.vitems)
        for (const WorkItem &w : l) v.emplace_back(-1, w.g, w.t);
    for (size_t i = 0; i < ll.fitems.size(); ++i)
        for (const WorkItem &w : ll.fitems[i]) v.emplace_back(ll.fshape[i].kind, w.g, w.t);
    std::sort(v.begin(), v.end());
    return v;
}

LaunchLists lists(const std::vector<GraphShape> &shapes, bool merge) {
    LaunchLists ll;
    std::vector<WorkItem> mids, highs, cols;
    for (size_t g = 0; g < shapes.size(); ++g) add_to_lists(ll, (int32_t)g, shapes[g], &mids, &highs, &cols);
    finish_lists(ll, mids, highs, cols, merge);
    return ll;
}

// launches of pairwise class (a, b); (0, 0) is the mixed launch
int count_pair(const LaunchLists &ll, int a, int b) {
    int n = 0;
    for (const FGroup &f : ll.fshape) n += f.kind == TK_PAIR && f.a == a && f.b == b;
    return n;
}

}  // namespace

int main() {
    // graphs of 2, 3 and 5 states, one with a hub (block-per-variable path),
    // one with a 3 x 4 pairwise factor (not square: stays in its own launch)
    Builder g2, g3, g5, gh;
    grid(g2, 9, 2);
    grid(g3, 12, 3);
    grid(g5, 7, 5);
    {
        const int hub = gh.var(3);
        const int t = gh.table(2);
        for (int i = 0; i < 300; ++i) gh.enumf({hub, gh.var(3)}, t);
        const int a = gh.var(3), b = gh.var(4);
        gh.enumf({a, b}, gh.table(2));
    }
    HostLayout L2, L3, L5, Lh;
    std::vector<GraphShape> shapes{shape_of(g2, L2), shape_of(g3, L3), shape_of(g5, L5), shape_of(gh, Lh)};

    const LaunchLists plain = lists(shapes, false), merged = lists(shapes, true);
    expect(items_of(plain) == items_of(merged), "merging lost, duplicated or moved work items");
    expect(count_pair(plain, 2, 2) == 1 && count_pair(plain, 3, 3) == 1 &&
               count_pair(plain, 5, 5) == 1,
           "unmerged lists keep one launch per square class");
    expect(plain.vbucket.size() > 1, "unmerged lists keep one variable launch per bucket");
    expect(count_pair(merged, 0, 0) == 1, "one mixed pairwise launch");
    int square = 0, other = 0;
    for (const FGroup &f : merged.fshape) {
        if (f.kind != TK_PAIR) continue;
        if (f.a == f.b && f.a >= 2 && f.a <= kPairStatesMax) ++square;
        if (f.a != f.b) ++other;
    }
    expect(square == 0, "no square class of 2..8 states left outside the mixed launch");
    expect(other == 1, "the 3 x 4 class keeps its own launch");
    expect(merged.vbucket.size() == 1 && merged.vbucket[0] == 8, "one variable launch of bucket 8");
    expect(merged.n_mid == plain.n_mid && merged.n_high == plain.n_high, "wavefront and block items unchanged");
    // the mixed launch's tiles are exactly the square tiles of every graph
    size_t sq_tiles = 0;
    for (size_t i = 0; i < plain.fshape.size(); ++i)
        if (plain.fshape[i].kind == TK_PAIR && plain.fshape[i].a == plain.fshape[i].b) sq_tiles += plain.fitems[i].size();
    for (size_t i = 0; i < merged.fshape.size(); ++i)
        if (merged.fshape[i].kind == TK_PAIR && merged.fshape[i].a == 0)
            expect(merged.fitems[i].size() == sq_tiles, "mixed launch holds every square tile");

    // one square class only: nothing to merge, the class keeps its launch
    std::vector<GraphShape> one{shapes[1], shapes[1]};
    const LaunchLists m1 = lists(one, true);
    expect(count_pair(m1, 3, 3) == 1 && count_pair(m1, 0, 0) == 0, "a single class is left alone");

    // a bucket above 8 keeps the variable launches apart
    Builder g9;
    grid(g9, 5, 9);
    HostLayout L9;
    std::vector<GraphShape> big{shapes[0], shape_of(g9, L9)};
    const LaunchLists mb = lists(big, true);
    expect(mb.vbucket.size() == 2, "buckets above 8 are not merged");
    expect(count_pair(mb, 2, 2) == 1, "a 9-state class does not join the mixed launch");
    expect(items_of(mb) == items_of(lists(big, false)), "work items kept with a large class");

    // two dense bipartite layers (70 x 80 and 70 x 100 binary units): their
    // hidden units form column groups.  The block-path items of the variable
    // launch are the groups of both graphs, then the single variables; group
    // position p holds group (p mod 8) * q + p / 8 of the graphs' groups in
    // order (q = n / 8; the last n mod 8 in place), so block p, on XCD p mod 8,
    // belongs to a run of consecutive groups.
    Builder b1, b2;
    auto layer = [](Builder &b, int nv, int nh) {
        for (int i = 0; i < nv + nh; ++i) b.var(2);
        const int t = b.table(2);
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < nh; ++j) b.enumf({i, nv + j}, t);
    };
    layer(b1, 70, 80);
    layer(b2, 70, 100);
    HostLayout Lb1, Lb2;
    std::vector<GraphShape> bip{shape_of(b1, Lb1), shape_of(b2, Lb2)};
    const LaunchLists lb = lists(bip, true);
    std::vector<WorkItem> groups;
    for (int32_t g = 0; g < 2; ++g)
        for (int32_t c : bip[g].cols) groups.push_back(WorkItem{g, c});
    const int64_t n = (int64_t)groups.size(), q = n / 8;
    expect(n >= 10 && !bip[0].cols.empty() && !bip[1].cols.empty(), "bipartite layers form column groups");
    expect(lb.n_high == (int32_t)(n + bip[0].highs.size() + bip[1].highs.size()), "block items: groups and singles");
    const std::vector<WorkItem> &v = lb.vitems[0];
    const size_t first = v.size() - (size_t)lb.n_high;
    bool order_ok = true;
    for (int64_t p = 0; p < n; ++p) {
        const WorkItem &want = groups[p < 8 * q ? (p % 8) * q + p / 8 : p];
        order_ok = order_ok && v[first + p].g == want.g && v[first + p].t == want.t;
    }
    size_t k = first + (size_t)n;
    for (int32_t g = 0; g < 2; ++g)
        for (int32_t h : bip[g].highs) {
            order_ok = order_ok && v[k].g == g && v[k].t == h;
            ++k;
        }
    expect(order_ok && k == v.size(), "column groups (swizzled), then single block-path variables");
    expect(items_of(lb) == items_of(lists(bip, false)), "work items kept with column groups");

    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("merge lists ok\n");
    return 0;
}
