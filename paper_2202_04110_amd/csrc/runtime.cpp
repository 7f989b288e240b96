// Internal runtime shared by the C-ABI and the serving loop (see runtime.h).
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

namespace lbp {

namespace {
thread_local std::string t_err;
}

int set_error(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

int hip_error(hipError_t e, const char *what) {
    return set_error(LBP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

const char *last_error() { return t_err.c_str(); }

bool valid_params(int32_t iters, float d, float T, std::string *why) {
    if (iters < 0) {
        *why = "iters < 0";
        return false;
    }
    if (!(d >= 0.0f && d <= 1.0f)) {
        *why = "damping outside [0, 1]";
        return false;
    }
    if (!(T >= 0.0f) || !std::isfinite(T)) {
        *why = "temperature must be finite and >= 0";
        return false;
    }
    return true;
}

// ------------------------------------------------------------ launch lists
void add_to_lists(LaunchLists &ll, int32_t gi, const GraphShape &s, std::vector<WorkItem> *mids,
                  std::vector<WorkItem> *highs, std::vector<WorkItem> *cols) {
    for (const VGroup &vg : s.vgroups) {
        size_t i = 0;
        while (i < ll.vbucket.size() && ll.vbucket[i] != vg.bucket) ++i;
        if (i == ll.vbucket.size()) {
            ll.vbucket.push_back(vg.bucket);
            ll.vitems.emplace_back();
        }
        for (int32_t t : vg.tiles) ll.vitems[i].push_back(WorkItem{gi, t});
    }
    for (int32_t h : s.mids) mids->push_back(WorkItem{gi, h});
    for (int32_t h : s.highs) highs->push_back(WorkItem{gi, h});
    for (int32_t h : s.cols) cols->push_back(WorkItem{gi, h});
    for (const FGroup &fg : s.fgroups) {
        size_t i = 0;
        while (i < ll.fshape.size() &&
               !(ll.fshape[i].kind == fg.kind && ll.fshape[i].a == fg.a && ll.fshape[i].b == fg.b))
            ++i;
        if (i == ll.fshape.size()) {
            FGroup sh;
            sh.kind = fg.kind;
            sh.a = fg.a;
            sh.b = fg.b;
            ll.fshape.push_back(sh);
            ll.fitems.emplace_back();
        }
        for (int32_t t : fg.tiles) ll.fitems[i].push_back(WorkItem{gi, t});
    }
}

namespace {
void merge_lists(LaunchLists &ll) {
    std::vector<size_t> sq;
    for (size_t i = 0; i < ll.fshape.size(); ++i) {
        const FGroup &f = ll.fshape[i];
        if (f.kind == TK_PAIR && f.a == f.b && f.a >= 2 && f.a <= kPairStatesMax) sq.push_back(i);
    }
    if (sq.size() > 1) {
        std::vector<FGroup> shape;
        std::vector<std::vector<WorkItem>> items;
        FGroup mixed;
        mixed.kind = TK_PAIR;
        mixed.a = mixed.b = 0;
        shape.push_back(mixed);
        items.emplace_back();
        size_t k = 0;
        for (size_t i = 0; i < ll.fshape.size(); ++i) {
            if (k < sq.size() && sq[k] == i) {
                items[0].insert(items[0].end(), ll.fitems[i].begin(), ll.fitems[i].end());
                ++k;
            } else {
                shape.push_back(ll.fshape[i]);
                items.push_back(std::move(ll.fitems[i]));
            }
        }
        ll.fshape = std::move(shape);
        ll.fitems = std::move(items);
    }
    bool small = ll.vbucket.size() > 1;
    int32_t top = 0;
    for (int32_t b : ll.vbucket) {
        small = small && b <= 8;
        top = std::max(top, b);
    }
    if (small) {
        std::vector<WorkItem> all;
        for (const auto &v : ll.vitems) all.insert(all.end(), v.begin(), v.end());
        ll.vbucket.assign(1, top);
        ll.vitems.assign(1, std::move(all));
    }
}
}  // namespace

void finish_lists(LaunchLists &ll, std::vector<WorkItem> &mids, std::vector<WorkItem> &highs,
                  std::vector<WorkItem> &cols, bool merge) {
    if (merge) merge_lists(ll);
    if (mids.empty() && highs.empty() && cols.empty()) return;
    if (ll.vbucket.empty()) {
        ll.vbucket.push_back(2);
        ll.vitems.emplace_back();
    }
    ll.n_mid = (int32_t)mids.size();
    ll.n_high = (int32_t)(cols.size() + highs.size());
    std::vector<WorkItem> &v = ll.vitems[0];
    v.insert(v.end(), mids.begin(), mids.end());
    // Block b of the variable launch takes block-path item b and runs on XCD
    // b mod 8 (workgroups go to the XCDs in turn).  Column group position p
    // holds group (p mod 8) * q + p / 8 (q = n / 8; the last n mod 8 keep
    // their place), so each XCD runs a run of consecutive groups: the groups
    // that read one cache line of edge rows then share that XCD's L2.
    const int64_t n = (int64_t)cols.size(), q = n / 8;
    for (int64_t p = 0; p < n; ++p) v.push_back(cols[p < 8 * q ? (p % 8) * q + p / 8 : p]);
    v.insert(v.end(), highs.begin(), highs.end());
}

size_t lists_bytes(const LaunchLists &ll) {
    size_t b = 0;
    for (const auto &v : ll.vitems) b += align256(std::max<size_t>(1, v.size()) * sizeof(WorkItem));
    for (const auto &v : ll.fitems) b += align256(std::max<size_t>(1, v.size()) * sizeof(WorkItem));
    return b;
}

// The lists' work items sit one 256-aligned run per launch: variable
// launches, then factor launches.
void describe_lists(const LaunchLists &ll, char *mem, std::vector<Launch> *vl, std::vector<Launch> *fl) {
    vl->clear();
    fl->clear();
    size_t off = 0;
    for (size_t i = 0; i < ll.vitems.size(); ++i) {
        const auto &v = ll.vitems[i];
        Launch L{-1, ll.vbucket[i], 0, 0, (WorkItem *)(mem + off)};
        L.n_mid = i == 0 ? ll.n_mid : 0;
        L.n_high = i == 0 ? ll.n_high : 0;
        L.n = (int32_t)v.size() - L.n_mid - L.n_high;
        vl->push_back(L);
        off += align256(std::max<size_t>(1, v.size()) * sizeof(WorkItem));
    }
    for (size_t i = 0; i < ll.fitems.size(); ++i) {
        const auto &v = ll.fitems[i];
        fl->push_back(Launch{ll.fshape[i].kind, ll.fshape[i].a, ll.fshape[i].b, (int32_t)v.size(),
                             (WorkItem *)(mem + off)});
        off += align256(std::max<size_t>(1, v.size()) * sizeof(WorkItem));
    }
}

void pack_lists(const LaunchLists &ll, char *host) {
    size_t off = 0;
    for (const auto *lists : {&ll.vitems, &ll.fitems})
        for (const auto &v : *lists) {
            if (!v.empty()) std::memcpy(host + off, v.data(), sizeof(WorkItem) * v.size());
            off += align256(std::max<size_t>(1, v.size()) * sizeof(WorkItem));
        }
}

hipError_t upload_lists(const LaunchLists &ll, char *mem, hipStream_t st, std::vector<Launch> *vl,
                        std::vector<Launch> *fl) {
    describe_lists(ll, mem, vl, fl);
    hipError_t e = hipSuccess;
    for (const auto *ls : {vl, fl})
        for (size_t i = 0; i < ls->size() && e == hipSuccess; ++i) {
            const Launch &L = (*ls)[i];
            const auto &v = ls == vl ? ll.vitems[i] : ll.fitems[i];
            if (!v.empty())
                e = hipMemcpyAsync(L.items, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice, st);
        }
    return e;
}

hipError_t launch_iteration(const DevGraph *gs, const std::vector<Launch> &vl, const std::vector<Launch> &fl,
                            const TParams &P, bool maxp, hipStream_t st, int phases) {
    hipError_t e = hipSuccess;
    if (phases & 1)
        for (const Launch &L : vl) {
            e = launch_belief(gs, L.items, L.n, L.n_mid, L.n_high, L.a, L.shape, st);
            if (e != hipSuccess) return e;
        }
    if (phases & 2)
        for (const Launch &L : fl) {
            switch (L.kind) {
            case TK_PAIR: e = launch_pair(gs, L.items, L.n, L.a, L.b, maxp, P, L.shape, st); break;
            case TK_LOGL: e = launch_logical(gs, L.items, L.n, false, maxp, P, L.shape, st); break;
            case TK_LOGW: e = launch_logical(gs, L.items, L.n, true, maxp, P, L.shape, st); break;
            default: e = launch_gen(gs, L.items, L.n, maxp, P, L.a, st); break;
            }
            if (e != hipSuccess) return e;
        }
    return e;
}

hipError_t launch_loop(const DevGraph *gs, const DevGraph *fused, const std::vector<Launch> &vl,
                       const std::vector<Launch> &fl, int32_t iters, const TParams &P, bool maxp, hipStream_t st,
                       int32_t fused_stride) {
    hipError_t e = hipSuccess;
    int32_t it = 0;
    if (fused)
        for (; it + 1 < iters && e == hipSuccess; it += 2)
            for (int h = 0; h < 2 && e == hipSuccess; ++h)
                for (const Launch &L : fl) {
                    e = launch_pair(fused + h * fused_stride, L.items, L.n, L.a, L.b, maxp, P, L.fshape, st, true);
                    if (e != hipSuccess) break;
                }
    for (; it < iters && e == hipSuccess; ++it) e = launch_iteration(gs, vl, fl, P, maxp, st);
    return e;
}

// ------------------------------------------------------------ captured loops
namespace {
constexpr size_t kMaxCachedLoops = 4;
}

void destroy_loops(std::vector<CachedLoop> &v) {
    for (CachedLoop &c : v) (void)hipGraphExecDestroy(c.exec);
    v.clear();
}

hipError_t run_loop(lbp_ctx *ctx, std::vector<CachedLoop> &cache, const DevGraph *gs, const DevGraph *fused,
                    const std::vector<Launch> &vl, const std::vector<Launch> &fl, int32_t iters, float d, float T,
                    int32_t fused_stride) {
    const TParams P = make_params(d, T);
    const bool maxp = T == 0.0f;
    const size_t per_iter = vl.size() + fl.size();
    if (!ctx->use_graphs || iters < 2 || per_iter == 0)
        return launch_loop(gs, fused, vl, fl, iters, P, maxp, ctx->stream, fused_stride);
    for (const CachedLoop &c : cache)
        if (c.iters == iters && c.d == d && c.T == T) return hipGraphLaunch(c.exec, ctx->stream);
    if (!ctx->capture) {
        hipError_t e = hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = launch_loop(gs, fused, vl, fl, iters, P, maxp, ctx->capture, fused_stride);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->capture, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return le != hipSuccess ? le : e;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (cache.size() >= kMaxCachedLoops) {
        (void)hipGraphExecDestroy(cache.front().exec);
        cache.erase(cache.begin());
    }
    cache.push_back(CachedLoop{iters, d, T, exec});
    return hipGraphLaunch(exec, ctx->stream);
}

// ------------------------------------------------------------ graph memory
namespace {

struct Piece {
    const void *src;
    size_t bytes;
    size_t off;
};

// The pieces of one graph's allocation in a fixed order (shared by the size
// query, the host image and the upload): the pieces with host data first,
// then the pieces that start as zeros.
struct GraphPieces {
    std::vector<Piece> p;
    size_t total = 0;
    size_t faff;
    bool raw = false;       // the image holds the raw evidence and tables; panels are scattered on the device
    size_t rev = 0, rlp = 0;
    size_t base = 0;        // device offset where the host image starts (after the raw potentials)
    size_t m, B, th, phi, ft, fvb, fvar, vt, ve, vns, hv, he, gc, gr, em, es, vs, vn, vx, fp, lp, fl, dg, q, map, items;
    size_t m2 = 0, fdg = 0;
    size_t data_end = 0;
    bool fused;
    LaunchLists ll;

    GraphPieces(const HostLayout &L, bool with_fused) : fused(with_fused && L.fusable) {
        auto add = [&](const void *src, size_t bytes) {
            p.push_back(Piece{src, bytes, total});
            total += align256(std::max<size_t>(bytes, 4));
            return p.size() - 1;
        };
        // A layout compiled with its panels carries them in the image.  One
        // compiled without them (the server's preparation threads) carries the
        // evidence as given instead, the tables as given come from a buffer
        // of their own, and graph_create scatters both into panels that
        // start as zeros: the device does the transpose.
        raw = L.theta_panel.size() != (size_t)L.VB || L.phi_panel.size() != (size_t)L.P;
        if (raw) {
            rlp = add(nullptr, sizeof(float) * L.Tn);  // copied from the caller's buffer, not the image
            base = total;
            rev = add(nullptr, sizeof(float) * L.VS);  // written by graph_fill_image
        } else {
            th = add(L.theta_panel.data(), sizeof(float) * L.VB);
            phi = add(L.phi_panel.data(), sizeof(float) * L.P);
        }
        ft = add(L.ftile.data(), sizeof(FTile) * L.ftile.size());
        fvb = add(L.fvb.data(), sizeof(int32_t) * L.fvb.size());
        fvar = add(L.fvar.data(), sizeof(int32_t) * L.fvar.size());
        faff = add(L.faff.data(), sizeof(int32_t) * L.faff.size());
        vt = add(L.vtile.data(), sizeof(VTile) * L.vtile.size());
        ve = add(L.vedge.data(), sizeof(int32_t) * L.vedge.size());
        vns = add(L.vns.data(), sizeof(int32_t) * L.vns.size());
        hv = add(L.hvar.data(), sizeof(HVar) * L.hvar.size());
        he = add(L.hedge.data(), sizeof(int32_t) * L.hedge.size());
        gc = add(L.gcls.data(), sizeof(GenClass) * L.gcls.size());
        gr = add(L.grows.data(), L.grows.size());
        em = add(L.edge_maddr.data(), sizeof(int32_t) * L.edge_maddr.size());
        es = add(L.es_off.data(), sizeof(int64_t) * L.es_off.size());
        vs = add(L.vs_off.data(), sizeof(int64_t) * L.vs_off.size());
        vn = add(L.vn.data(), sizeof(int32_t) * L.vn.size());
        vx = add(L.vext.data(), sizeof(int32_t) * L.vext.size());
        fp = add(L.fac_phi.data(), sizeof(int32_t) * L.fac_phi.size());
        lp = add(L.lp_off.data(), sizeof(int64_t) * L.lp_off.size());
        GraphShape s{L.fgroups, L.vgroups, L.mids, L.highs, L.cols};
        std::vector<WorkItem> mids, highs, cols;
        add_to_lists(ll, 0, s, &mids, &highs, &cols);
        finish_lists(ll, mids, highs, cols);
        items = add(nullptr, lists_bytes(ll));  // packed by pack_lists
        dg = add(nullptr, sizeof(DevGraph));    // written into the image by graph_create
        data_end = total;  // everything above is copied from the host image, everything below starts zero
        m = add(nullptr, sizeof(float) * L.M);
        B = add(nullptr, sizeof(float) * L.VB);
        fl = add(nullptr, sizeof(int32_t) * 4);
        if (raw) {
            th = add(nullptr, sizeof(float) * L.VB);
            phi = add(nullptr, sizeof(float) * L.P);
        }
        q = add(nullptr, sizeof(float) * L.VS);
        map = add(nullptr, sizeof(int32_t) * L.V);
        if (fused) {
            m2 = add(nullptr, sizeof(float) * L.M);
            fdg = add(nullptr, sizeof(DevGraph) * 2);
        }
    }
};

}  // namespace

size_t graph_device_bytes(const HostLayout &L, bool with_fused) { return GraphPieces(L, with_fused).total; }

size_t graph_image_bytes(const HostLayout &L) {
    GraphPieces gp(L, false);
    return gp.data_end - gp.base;
}

int graph_fill_image(const HostLayout &L, char *image, const lbp_graph_desc *d) {
    GraphPieces gp(L, false);
    // pieces are placed by device offset; the image starts at gp.base (every
    // piece written here lies at or above it)
    auto at = [&](size_t off) { return image + (off - gp.base); };
    for (const Piece &p : gp.p)
        if (p.src && p.bytes) std::memcpy(at(p.off), p.src, p.bytes);
    pack_lists(gp.ll, at(gp.p[gp.items].off));
    if (!gp.raw) return LBP_OK;
    // the evidence as given (graph_create scatters it into its panel)
    if (!d) return set_error(LBP_E_INVALID, "graph image: the layout has no panels and no description was given");
    float *ev = (float *)at(gp.p[gp.rev].off);
    if (d->evidence) std::memcpy(ev, d->evidence, sizeof(float) * L.VS);
    else std::memset(ev, 0, sizeof(float) * L.VS);
    return LBP_OK;
}

int graph_create(lbp_ctx *ctx, const HostLayout &L, bool with_fused, char *mem, hipStream_t st, lbp_graph **out,
                 char *image, bool wait, const float *raw_lp) {
    lbp_graph *g = nullptr;
    char *own_image = nullptr;  // built here when the caller brings none
    try {
        GraphPieces gp(L, with_fused);
        g = new lbp_graph;
        g->ctx = ctx;
        if (mem) {
            g->dmem = mem;
            g->owns_memory = false;
        } else {
            hipError_t e = hipMalloc((void **)&g->dmem, gp.total);
            if (e != hipSuccess) {
                delete g;
                (void)hipGetLastError();
                return set_error(LBP_E_OOM, "device allocation of " + std::to_string(gp.total) + " bytes failed");
            }
        }
        g->dbytes = gp.total;
        auto ptr = [&](size_t i) { return (void *)(g->dmem + gp.p[i].off); };
        if (gp.raw && (!image || (L.Tn > 0 && !raw_lp))) {
            if (g->owns_memory) (void)hipFree(g->dmem);
            delete g;
            return set_error(LBP_E_INVALID, "graph_create: a layout without panels needs its image and potentials");
        }
        if (!image) {
            wait = true;  // the image built here is freed before returning
            own_image = (char *)panel_alloc(gp.data_end);
            if (!own_image) throw std::bad_alloc();
            graph_fill_image(L, own_image, nullptr);  // compiled with its panels: cannot fail
            image = own_image;
        }
        DevGraph &h = g->host;
        h.m = (float *)ptr(gp.m);
        h.mo = h.m;
        h.B = (float *)ptr(gp.B);
        h.theta = (float *)ptr(gp.th);
        h.phi = (float *)ptr(gp.phi);
        h.ftile = (const FTile *)ptr(gp.ft);
        h.fvb = (const int32_t *)ptr(gp.fvb);
        h.fvar = (const int32_t *)ptr(gp.fvar);
        h.faff = (const int32_t *)ptr(gp.faff);
        h.vtile = (const VTile *)ptr(gp.vt);
        h.vedge = (const int32_t *)ptr(gp.ve);
        h.vns = (const int32_t *)ptr(gp.vns);
        h.hvar = (const HVar *)ptr(gp.hv);
        h.hedge = (const int32_t *)ptr(gp.he);
        h.gcls = (const GenClass *)ptr(gp.gc);
        h.grows = (const uint8_t *)ptr(gp.gr);
        h.edge_maddr = (const int32_t *)ptr(gp.em);
        h.es_off = (const int64_t *)ptr(gp.es);
        h.vs_off = (const int64_t *)ptr(gp.vs);
        h.vn = (const int32_t *)ptr(gp.vn);
        h.vext = L.vext.empty() ? nullptr : (const int32_t *)ptr(gp.vx);
        h.fac_phi = (const int32_t *)ptr(gp.fp);
        h.lp_off = (const int64_t *)ptr(gp.lp);
        h.flag = (int32_t *)ptr(gp.fl);
        h.V = (int32_t)L.V;
        h.E = (int32_t)L.E;
        h.F = (int32_t)L.F;
        h.zero_addr = L.zero_addr;
        h.raw_msgs = 0;
        g->dgraph = (DevGraph *)ptr(gp.dg);
        g->q_tmp = (float *)ptr(gp.q);
        g->map_tmp = (int32_t *)ptr(gp.map);
        // the descriptor travels in the image: one copy of every host piece
        // (a single DMA when the image is page-locked), one fill for
        // messages, beliefs, flag and scratch
        std::memcpy(image + (gp.p[gp.dg].off - gp.base), &g->host, sizeof(DevGraph));
        hipError_t e = hipSuccess;
        if (gp.raw && L.Tn > 0)
            e = hipMemcpyAsync(ptr(gp.rlp), raw_lp, sizeof(float) * L.Tn, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->dmem + gp.base, image, gp.data_end - gp.base, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemsetAsync(g->dmem + gp.data_end, 0, gp.total - gp.data_end, st);
        if (gp.raw && e == hipSuccess) {  // panels from the raw evidence and tables of the image
            e = launch_evidence_in(g->dgraph, (int)L.V, (const float *)ptr(gp.rev), st);
            if (e == hipSuccess) e = launch_logpot_in(g->dgraph, (int)L.F, (const float *)ptr(gp.rlp), st);
        }
        DevGraph fv[2];
        if (gp.fused) {
            float *m2 = (float *)ptr(gp.m2);
            fv[0] = g->host;
            fv[0].mo = m2;
            fv[1] = g->host;
            fv[1].m = m2;
            fv[1].mo = g->host.m;
            g->fused = (DevGraph *)ptr(gp.fdg);
            g->m2 = m2;
            if (e == hipSuccess) e = hipMemcpyAsync(g->fused, fv, sizeof(fv), hipMemcpyHostToDevice, st);
        }
        describe_lists(gp.ll, (char *)ptr(gp.items), &g->vl, &g->fl);
        // the host image and the descriptors must outlive the copies (the
        // descriptors live in g; without wait, the caller keeps the image)
        if (e == hipSuccess && (wait || gp.fused)) e = hipStreamSynchronize(st);
        if (e != hipSuccess) (void)hipStreamSynchronize(st);  // no copy may still read an image
        panel_free(own_image);
        own_image = nullptr;
        if (e != hipSuccess) {
            if (g->owns_memory) (void)hipFree(g->dmem);
            delete g;
            return hip_error(e, "graph upload");
        }
        g->shape = GraphShape{L.fgroups, L.vgroups, L.mids, L.highs, L.cols};
        for (const FGroup &fg : L.fgroups)
            if (fg.kind == TK_LOGL || fg.kind == TK_LOGW) g->has_logical = true;
        g->V = L.V; g->VS = L.VS; g->F = L.F; g->E = L.E; g->ES = L.ES; g->Tn = L.Tn;
        g->M = L.M; g->VB = L.VB; g->P = L.P;
        g->nvt = (int32_t)L.vtile.size();
        g->resident_ok = make_solve_plan(g->vl, g->fl, L, solve_lds_limit(ctx->device) / 4, &g->plan);
        *out = g;
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        panel_free(own_image);
        if (g) {
            if (g->dmem && g->owns_memory) (void)hipFree(g->dmem);
            delete g;
        }
        return set_error(LBP_E_OOM, "host allocation failed");
    }
}

bool make_solve_plan(const std::vector<Launch> &vl, const std::vector<Launch> &fl, const HostLayout &L,
                     int64_t limit_words, SolvePlan *plan) {
    static_assert(sizeof(VTile) == 16 && sizeof(FTile) == 32 && sizeof(HVar) == 16, "4-byte-word structs");
    const int64_t w[SA_COUNT] = {L.M, L.VB, (int64_t)L.vedge.size(), (int64_t)L.fvb.size(), (int64_t)L.hedge.size(),
                                 (int64_t)L.vns.size(), 4 * (int64_t)L.vtile.size(), 8 * (int64_t)L.ftile.size(),
                                 4 * (int64_t)L.hvar.size(), L.VB, L.P};
    if (L.M <= 0 || L.VB <= 0 || solve_words_aligned(w[SA_M]) + solve_words_aligned(w[SA_B]) > limit_words ||
        vl.size() + fl.size() > (size_t)kSolveLaunchesMax)
        return false;
    SolvePlan p;
    int64_t used = 0;
    for (int a = 0; a < SA_COUNT; ++a) {
        p.words[a] = (int32_t)w[a];
        if (used + solve_words_aligned(w[a]) <= limit_words) {
            p.lds_mask |= 1u << a;
            used += solve_words_aligned(w[a]);
        }
    }
    p.lds_words = (int32_t)used;
    for (const Launch &x : vl) {
        if (x.n_high != 0) return false;
        p.l[p.nv++] = SolveLaunch{-1, x.a, 0, x.n, x.n_mid, 0, x.items};
    }
    for (const Launch &x : fl) {
        if (x.kind != TK_PAIR && x.kind != TK_LOGL) return false;
        p.l[p.nv + p.nf++] = SolveLaunch{x.kind, x.a, x.b, x.n, 0, 0, x.items};
    }
    *plan = p;
    return true;
}

void graph_destroy(lbp_graph *g) {
    if (!g) return;
    destroy_loops(g->loops);
    if (g->conv) (void)hipFree(g->conv);
    if (g->adj.dmem && g->adj.owns_memory) (void)hipFree(g->adj.dmem);
    if (g->owns_memory) (void)hipFree(g->dmem);
    delete g;
}

int graph_readout(lbp_graph *g, float *q, int normalized, int32_t *map, bool on_device, hipStream_t st) {
    const TParams P = make_params(0.5f, g->last_T);
    const bool maxp = g->last_T == 0.0f;
    hipError_t e = launch_iteration(g->dgraph, g->vl, g->fl, P, maxp, st, 1);
    if (e != hipSuccess) return hip_error(e, "belief launch");
    float *qd = q ? (on_device ? q : g->q_tmp) : nullptr;
    int32_t *md = map ? (on_device ? map : g->map_tmp) : nullptr;
    HIP_TRY(launch_readout(g->dgraph, g->nvt, maxp, P, qd, normalized, md, st));
    if (on_device) return LBP_OK;
    if (q) HIP_TRY(hipMemcpyAsync(q, g->q_tmp, sizeof(float) * g->VS, hipMemcpyDeviceToHost, st));
    if (map) HIP_TRY(hipMemcpyAsync(map, g->map_tmp, sizeof(int32_t) * g->V, hipMemcpyDeviceToHost, st));
    return LBP_OK;
}

// ------------------------------------------------------------ reverse sweep
namespace {

struct AdjLayout {
    size_t ck, seg, A, nb, Bb, Bt, z, tb, pb, v, total;
    AdjLayout(size_t M, size_t VB, size_t P, int32_t nseg, int32_t k) {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off += align256(std::max<size_t>(bytes, 4));
            return o;
        };
        ck = take(sizeof(float) * M * std::max(nseg, 1));
        seg = take(sizeof(float) * M * k);
        A = take(sizeof(float) * M);
        nb = take(sizeof(float) * M);
        Bb = take(sizeof(float) * VB);
        Bt = take(sizeof(float) * VB);
        z = take(sizeof(float) * VB);
        tb = take(sizeof(float) * VB);
        pb = take(sizeof(float) * P);
        v = take(sizeof(DevGraph) * (k + 2));
        total = off;
    }
};

void record_shape(int32_t iters, int32_t ckpt_every, int32_t *k, int32_t *nseg) {
    *k = std::min<int32_t>(ckpt_every, std::max<int32_t>(iters, 1));
    *nseg = (iters + *k - 1) / *k;
}

}  // namespace

size_t adjoint_bytes(int64_t M, int64_t VB, int64_t P, int32_t iters, int32_t ckpt_every) {
    int32_t k, nseg;
    record_shape(iters, ckpt_every, &k, &nseg);
    return AdjLayout((size_t)M, (size_t)VB, (size_t)P, nseg, k).total;
}

int adjoint_prepare(lbp_graph *g, int32_t iters, float d, float T, int32_t ckpt_every, char *mem, hipStream_t st,
                    std::vector<DevGraph> *staging) {
    auto &J = g->adj;
    J.valid = false;
    int32_t k, nseg;
    record_shape(iters, ckpt_every, &k, &nseg);
    const AdjLayout al((size_t)g->M, (size_t)g->VB, (size_t)g->P, nseg, k);
    if (mem) {
        if (J.dmem && J.owns_memory) {
            HIP_TRY(hipStreamSynchronize(st));
            (void)hipFree(J.dmem);
        }
        J.dmem = mem;
        J.bytes = al.total;
        J.owns_memory = false;
    } else if (!J.owns_memory || al.total > J.bytes) {
        if (J.dmem && J.owns_memory) {
            HIP_TRY(hipStreamSynchronize(st));
            (void)hipFree(J.dmem);
        }
        J.dmem = nullptr;
        J.bytes = 0;
        J.owns_memory = true;
        hipError_t e = hipMalloc((void **)&J.dmem, al.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            J.dmem = nullptr;
            return set_error(LBP_E_OOM, "adjoint workspace of " + std::to_string(al.total) + " bytes");
        }
        J.bytes = al.total;
    }
    const size_t M = (size_t)g->M, VB = (size_t)g->VB;
    J.ckpt = (float *)(J.dmem + al.ck);
    J.seg = (float *)(J.dmem + al.seg);
    J.A = (float *)(J.dmem + al.A);
    J.nbar = (float *)(J.dmem + al.nb);
    J.Bbar = (float *)(J.dmem + al.Bb);
    J.Bt = (float *)(J.dmem + al.Bt);
    J.zeros = (float *)(J.dmem + al.z);
    J.thetabar = (float *)(J.dmem + al.tb);
    J.phibar = (float *)(J.dmem + al.pb);
    J.views = (DevGraph *)(J.dmem + al.v);
    // zero panels of the iterate buffers and of nbar must read as zero
    HIP_TRY(hipMemsetAsync(J.seg, 0, sizeof(float) * M * k, st));
    HIP_TRY(hipMemsetAsync(J.nbar, 0, sizeof(float) * M, st));
    HIP_TRY(hipMemsetAsync(J.zeros, 0, sizeof(float) * VB, st));
    std::vector<DevGraph> local;
    std::vector<DevGraph> &views = staging ? *staging : local;
    views.assign(k + 2, g->host);
    for (int32_t j = 0; j < k; ++j) {
        views[j].m = J.seg + M * j;
        views[j].mo = J.seg + M * std::min(j + 1, k - 1);
        views[j].B = J.Bt;
    }
    views[k].B = J.Bt;
    views[k + 1].m = J.nbar;
    views[k + 1].mo = J.nbar;
    views[k + 1].raw_msgs = 1;  // adjoint sums, one state per panel row
    views[k + 1].theta = J.zeros;
    views[k + 1].B = J.Bbar;
    HIP_TRY(hipMemcpyAsync(J.views, views.data(), sizeof(DevGraph) * (k + 2), hipMemcpyHostToDevice, st));
    if (!staging) HIP_TRY(hipStreamSynchronize(st));  // the local staging must outlive its copy
    J.iters = iters;
    J.k = k;
    J.nseg = nseg;
    J.d = d;
    J.T = T;
    return LBP_OK;
}

int adjoint_checkpoint(lbp_graph *g, int32_t seg, hipStream_t st) {
    auto &J = g->adj;
    HIP_TRY(hipMemcpyAsync(J.ckpt + (size_t)g->M * seg, g->host.m, sizeof(float) * g->M, hipMemcpyDeviceToDevice, st));
    return LBP_OK;
}

void adjoint_finish_record(lbp_graph *g) {
    g->adj.valid = true;
    g->adj.version = g->version;
}

int adjoint_backward(lbp_graph *g, const float *grad_q, float *grad_logpot, float *grad_evidence, hipStream_t st) {
    auto &J = g->adj;
    const TParams P = make_params(J.d, J.T);
    const int64_t M = g->M;
    const int k = J.k;
    AdjBufs B{J.A, J.nbar, J.Bbar, J.phibar};
    HIP_TRY(hipMemsetAsync(J.A, 0, sizeof(float) * M, st));
    HIP_TRY(hipMemsetAsync(J.phibar, 0, sizeof(float) * g->P, st));
    // read-out adjoint at the recorded final iterate (the graph's messages)
    hipError_t e = launch_iteration(J.views + k, g->vl, g->fl, P, false, st, 1);
    if (e == hipSuccess) e = launch_readout_adj(J.views + k, g->nvt, P, grad_q, J.Bbar, J.thetabar, st);
    for (int32_t sidx = J.nseg - 1; sidx >= 0 && e == hipSuccess; --sidx) {
        const int32_t len = std::min(k, J.iters - sidx * k);
        e = hipMemcpyAsync(J.seg, J.ckpt + M * sidx, sizeof(float) * M, hipMemcpyDeviceToDevice, st);
        for (int32_t j = 0; j + 1 < len && e == hipSuccess; ++j)
            e = launch_iteration(J.views + j, g->vl, g->fl, P, false, st, 3);
        for (int32_t j = len - 1; j >= 0 && e == hipSuccess; --j) {
            e = launch_iteration(J.views + j, g->vl, g->fl, P, false, st, 1);  // B_t
            for (const Launch &L : g->fl) {
                if (e != hipSuccess) break;
                if (L.kind == TK_PAIR) e = launch_pair_adj(J.views + j, L.items, L.n, L.a, L.b, P, B, st);
                else e = launch_gen_adj(J.views + j, L.items, L.n, P, B, st);
            }
            if (e == hipSuccess) e = launch_iteration(J.views + k + 1, g->vl, g->fl, P, false, st, 1);  // Bbar_t
            if (e == hipSuccess) e = launch_accumulate(J.thetabar, J.Bbar, g->VB, st);
        }
    }
    if (e == hipSuccess) e = launch_logpot_out(g->dgraph, (int)g->F, J.phibar, grad_logpot, st);
    if (e == hipSuccess && grad_evidence) e = launch_evidence_out(g->dgraph, (int)g->V, J.thetabar, grad_evidence, st);
    if (e != hipSuccess) return hip_error(e, "backward launch");
    return LBP_OK;
}

}  // namespace lbp
