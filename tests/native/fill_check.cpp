// Host-only test of the potential panels (fill_panels): every panel entry
// equals the table value of the factor in that lane at that configuration,
// lanes without a factor hold zero, and a NaN or infinity anywhere in the
// tables is rejected.  Covers full and partial 16-lane blocks, dense
// pairwise classes whose configuration counts are and are not multiples of
// 4, and a three-way class.  Built against liblbp.so and run by
// tests/test_fill_check.py.
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <limits>
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

// Compiles b without panels, fills them, and compares each entry with the
// table it came from.
void check(const char *name, Builder &b) {
    HostLayout L;
    std::string err;
    const lbp_graph_desc *d = b.desc();
    int rc = compile_desc(d, &L, &err, false);
    expect(rc == LBP_OK, std::string(name) + ": compile: " + err);
    if (rc != LBP_OK) return;
    std::vector<float> theta(L.VB, -1.0f), phi(L.P, -1.0f);
    rc = fill_panels(d, L, theta.data(), phi.data(), &err);
    expect(rc == LBP_OK, std::string(name) + ": fill: " + err);
    long checked = 0, bad = 0;
    for (size_t t = 0; t < L.ftile.size(); ++t) {
        const FTile &ft = L.ftile[t];
        if (ft.kind != TK_PAIR && ft.kind != TK_GEN) continue;
        const int32_t ncfg = ft.kind == TK_PAIR ? ft.a * ft.b : L.gcls[ft.a].ncfg;
        for (int32_t l = 0; l < kLanes; ++l) {
            const int32_t f = L.tile_fac[t * kLanes + l];
            for (int32_t c = 0; c < ncfg; ++c) {
                const float want = f >= 0 ? d->log_potentials[L.lp_off[f] + c] : 0.0f;
                const float got = phi[ft.phi_off + (int64_t)c * kLanes + l];
                bad += got != want;
                ++checked;
            }
        }
    }
    expect(bad == 0, std::string(name) + ": " + std::to_string(bad) + " of " + std::to_string(checked) +
                         " panel entries differ from their tables");
    // a NaN, then an infinity, in the last factor's table
    for (float x : {std::numeric_limits<float>::quiet_NaN(), -std::numeric_limits<float>::infinity()}) {
        const float keep = b.lp.back();
        b.lp.back() = x;
        std::string e;
        const int r = fill_panels(b.desc(), L, theta.data(), phi.data(), &e);
        expect(r == LBP_E_INVALID && e.find("not finite") != std::string::npos,
               std::string(name) + ": non-finite table value accepted: " + e);
        b.lp.back() = keep;
    }
    std::printf("%s: %ld panel entries checked\n", name, checked);
}

void grid(Builder &b, int side, int n) {
    const int v0 = (int)b.ns.size();
    for (int i = 0; i < side * side; ++i) b.var(n);
    const int t = b.table(2);
    for (int r = 0; r < side; ++r)
        for (int c = 0; c + 1 < side; ++c) b.enumf({v0 + r * side + c, v0 + r * side + c + 1}, t);
    for (int r = 0; r + 1 < side; ++r)
        for (int c = 0; c < side; ++c) b.enumf({v0 + r * side + c, v0 + (r + 1) * side + c}, t);
}

}  // namespace

int main() {
    // 9 configurations (not a multiple of 4), the last tile partial
    Builder a;
    grid(a, 11, 3);
    check("grid 11x11, 3 states", a);
    // 16 configurations, full tiles and a partial one
    Builder b;
    grid(b, 13, 4);
    check("grid 13x13, 4 states", b);
    // several classes at once: 2 x 5 pairs (10 configurations) and a
    // three-way class (2 x 3 x 3 = 18 configurations)
    Builder c;
    std::vector<int> v2, v5, v3;
    for (int i = 0; i < 70; ++i) v2.push_back(c.var(2));
    for (int i = 0; i < 70; ++i) v5.push_back(c.var(5));
    for (int i = 0; i < 40; ++i) v3.push_back(c.var(3));
    const int tp = c.table(2), t3 = c.table(3);
    for (int i = 0; i < 70; ++i) c.enumf({v2[i], v5[(i * 7) % 70]}, tp);
    for (int i = 0; i + 1 < 40; ++i) c.enumf({v2[i], v3[i], v3[i + 1]}, t3);
    check("mixed classes", c);

    // the submission-time copy of the potentials: every value copied bit for
    // bit (signed zeros, denormals, the largest finite values included) and
    // the first NaN or infinity reported, wherever it falls in its block
    {
        const int64_t n = 3 * 4096 + 77;
        std::vector<float> src(n), dst(n);
        for (int64_t i = 0; i < n; ++i) src[i] = (float)((i * 37) % 1001) * 0.25f - 100.0f;
        src[5] = -0.0f;
        src[9] = 1e-40f;
        src[11] = 3.4e38f;
        src[12] = -3.4e38f;
        int64_t r = copy_check_finite(dst.data(), src.data(), n);
        expect(r == -1, "finite copy: no index");
        expect(std::memcmp(dst.data(), src.data(), sizeof(float) * n) == 0, "finite copy: bitwise");
        const float bad[3] = {std::numeric_limits<float>::quiet_NaN(), std::numeric_limits<float>::infinity(),
                              -std::numeric_limits<float>::infinity()};
        const int64_t at[4] = {0, 4095, 4096, n - 1};
        for (float b : bad)
            for (int64_t i : at) {
                std::vector<float> s2(src);
                s2[i] = b;
                if (i + 100 < n) s2[i + 100] = b;  // a later one is not the first
                std::fill(dst.begin(), dst.end(), 7.0f);
                r = copy_check_finite(dst.data(), s2.data(), n);
                expect(r == i, "non-finite copy: first index " + std::to_string(i));
                expect(std::memcmp(dst.data(), s2.data(), sizeof(float) * n) == 0, "non-finite copy: bitwise");
            }
        expect(copy_check_finite(dst.data(), src.data(), 0) == -1, "empty copy");
    }
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("fill check ok\n");
    return 0;
}
