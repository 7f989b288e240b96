// C-ABI of liblbp.so (declared in include/lbp.h): contexts, graph upload,
// iteration driver, read-out, state exchange and batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbp.h"
#include "compile.h"
#include "kernels.h"

using namespace lbp;

namespace {

thread_local std::string t_err;

int fail(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(LBP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

// A set of work items launched by one kernel.
struct Launch {
    int32_t kind;  // -1 variable phase, TK_* factor kernels
    int32_t a, b;  // variable phase: state bucket; PAIR: slot state counts
    int32_t n;     // items (variable phase: low tiles)
    WorkItem *items;  // device
    int32_t n_mid = 0, n_high = 0;  // variable phase: wavefront- and block-per-variable items after the tiles
};

// Variable-phase launches: one per state bucket of the low tiles; the first
// also carries every mid and high variable.
struct VarWork {
    std::vector<int32_t> buckets;
    std::vector<std::vector<WorkItem>> items;  // per bucket: tiles, then (first only) mids, highs
    int32_t n_mid = 0, n_high = 0;
};

void add_var_work(VarWork &vw, int32_t gi, const std::vector<VGroup> &vgroups, const std::vector<int32_t> &mids,
                  const std::vector<int32_t> &highs, std::vector<WorkItem> *mid_out, std::vector<WorkItem> *high_out) {
    for (const VGroup &vg : vgroups) {
        size_t i = 0;
        while (i < vw.buckets.size() && vw.buckets[i] != vg.bucket) ++i;
        if (i == vw.buckets.size()) {
            vw.buckets.push_back(vg.bucket);
            vw.items.emplace_back();
        }
        for (int32_t t : vg.tiles) vw.items[i].push_back(WorkItem{gi, t});
    }
    for (int32_t h : mids) mid_out->push_back(WorkItem{gi, h});
    for (int32_t h : highs) high_out->push_back(WorkItem{gi, h});
}

// Appends mids/highs to the first bucket's list (creating one if needed).
void finish_var_work(VarWork &vw, std::vector<WorkItem> &mids, std::vector<WorkItem> &highs) {
    if (mids.empty() && highs.empty()) return;
    if (vw.buckets.empty()) {
        vw.buckets.push_back(2);
        vw.items.emplace_back();
    }
    vw.n_mid = (int32_t)mids.size();
    vw.n_high = (int32_t)highs.size();
    vw.items[0].insert(vw.items[0].end(), mids.begin(), mids.end());
    vw.items[0].insert(vw.items[0].end(), highs.begin(), highs.end());
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

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

// Launches one iteration (variable phase then factor phase) of every launch
// group over the graph array `gs`.
hipError_t launch_iteration(const DevGraph *gs, const std::vector<Launch> &vl, const std::vector<Launch> &fl,
                            const TParams &P, bool maxp, hipStream_t st, int phases = 3) {
    hipError_t e = hipSuccess;
    if (phases & 1)
        for (const Launch &L : vl) {
            e = launch_belief(gs, L.items, L.n, L.n_mid, L.n_high, L.a, st);
            if (e != hipSuccess) return e;
        }
    if (phases & 2)
        for (const Launch &L : fl) {
            switch (L.kind) {
            case TK_PAIR: e = launch_pair(gs, L.items, L.n, L.a, L.b, maxp, P, st); break;
            case TK_LOGL: e = launch_logical(gs, L.items, L.n, false, maxp, P, st); break;
            case TK_LOGW: e = launch_logical(gs, L.items, L.n, true, maxp, P, st); break;
            default: e = launch_gen(gs, L.items, L.n, maxp, P, st); break;
            }
            if (e != hipSuccess) return e;
        }
    return e;
}

}  // namespace

struct lbp_ctx {
    int device;
    hipStream_t stream;          // the caller's stream (borrowed)
    hipStream_t capture = nullptr;  // private stream used only to record launch graphs
    bool use_graphs = true;
};

namespace {

// A captured fixed-iteration loop, replayed with hipGraphLaunch.
struct CachedLoop {
    int32_t iters;
    float d, T;
    hipGraphExec_t exec;
};

constexpr size_t kMaxCachedLoops = 4;

void destroy_loops(std::vector<CachedLoop> &v) {
    for (CachedLoop &c : v) (void)hipGraphExecDestroy(c.exec);
    v.clear();
}

// Runs `iters` iterations on ctx->stream: through a cached captured graph
// when enabled (the kernels and their arguments are the same as eager
// launches), else by launching each kernel.
hipError_t run_loop(lbp_ctx *ctx, std::vector<CachedLoop> &cache, const DevGraph *gs, const std::vector<Launch> &vl,
                    const std::vector<Launch> &fl, int32_t iters, float d, float T) {
    const TParams P = make_params(d, T);
    const bool maxp = T == 0.0f;
    const size_t per_iter = vl.size() + fl.size();
    if (!ctx->use_graphs || iters < 2 || per_iter == 0) {
        for (int32_t it = 0; it < iters; ++it) {
            hipError_t e = launch_iteration(gs, vl, fl, P, maxp, ctx->stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    for (const CachedLoop &c : cache)
        if (c.iters == iters && c.d == d && c.T == T) return hipGraphLaunch(c.exec, ctx->stream);
    if (!ctx->capture) {
        hipError_t e = hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int32_t it = 0; it < iters && le == hipSuccess; ++it)
        le = launch_iteration(gs, vl, fl, P, maxp, ctx->capture);
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

}  // namespace

struct lbp_graph {
    lbp_ctx *ctx = nullptr;
    int64_t V = 0, VS = 0, F = 0, E = 0, ES = 0, Tn = 0, M = 0, VB = 0, P = 0;
    int32_t nvt = 0;
    char *dmem = nullptr;
    size_t dbytes = 0;
    DevGraph host{};              // device pointers, host copy
    DevGraph *dgraph = nullptr;   // device copy
    float *q_tmp = nullptr;       // VS
    int32_t *map_tmp = nullptr;   // V
    std::vector<Launch> vl, fl;   // variable-phase and factor-phase launches
    std::vector<FGroup> fgroups;  // shapes (batches merge by shape)
    std::vector<VGroup> vgroups;
    std::vector<int32_t> mids, highs;
    float last_T = 0.0f;
    std::vector<CachedLoop> loops;
    bool has_logical = false;
    uint64_t version = 0;  // bumped by every call that changes messages or inputs
    // reverse-sweep workspace and the record it belongs to
    struct Adjoint {
        bool valid = false;
        uint64_t version = 0;
        int32_t iters = 0, k = 0, nseg = 0;
        float d = 0.0f, T = 0.0f;
        char *dmem = nullptr;
        size_t bytes = 0;
        float *ckpt = nullptr, *seg = nullptr, *A = nullptr, *nbar = nullptr, *Bbar = nullptr, *Bt = nullptr,
              *zeros = nullptr, *thetabar = nullptr, *phibar = nullptr;
        DevGraph *views = nullptr;  // [0, k): iterates in seg; [k]: current messages; [k+1]: adjoint view
    } adj;
};

struct lbp_batch {
    lbp_ctx *ctx = nullptr;
    std::vector<lbp_graph *> graphs;
    char *dmem = nullptr;
    DevGraph *dgraphs = nullptr;
    std::vector<Launch> vl, fl;
    std::vector<CachedLoop> loops;
};

extern "C" {

const char *lbp_last_error(void) { return t_err.c_str(); }

int lbp_validate(const lbp_graph_desc *desc, int64_t sizes_out[6]) {
    try {
        std::string err;
        int64_t sz[6];
        int rc = validate_desc(desc, sz, &err);
        if (rc != LBP_OK) return fail(rc, err);
        if (sizes_out) std::memcpy(sizes_out, sz, sizeof(sz));
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        return fail(LBP_E_OOM, "host allocation failed");
    }
}

int lbp_check_layout(const lbp_graph_desc *desc, int64_t info_out[4]) {
    try {
        HostLayout L;
        std::string err;
        int rc = compile_desc(desc, &L, &err);
        if (rc == LBP_OK) rc = check_layout(L, &err);
        if (rc != LBP_OK) return fail(rc, err);
        if (info_out) {
            info_out[0] = L.M;
            info_out[1] = L.VB;
            info_out[2] = L.P;
            info_out[3] = (int64_t)L.ftile.size();
        }
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        return fail(LBP_E_OOM, "host allocation failed");
    }
}

int lbp_ctx_create(int device, void *hip_stream, lbp_ctx **out) {
    if (!out) return fail(LBP_E_INVALID, "out is NULL");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(LBP_E_INVALID, "device index out of range");
    HIP_TRY(hipSetDevice(device));
    lbp_ctx *c = new (std::nothrow) lbp_ctx;
    if (!c) return fail(LBP_E_OOM, "host allocation failed");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    const char *env = getenv("LBP_NO_GRAPHS");
    c->use_graphs = !(env && env[0] && env[0] != '0');
    *out = c;
    return LBP_OK;
}

int lbp_ctx_set_stream(lbp_ctx *ctx, void *hip_stream) {
    if (!ctx) return fail(LBP_E_INVALID, "ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return LBP_OK;
}

int lbp_ctx_synchronize(lbp_ctx *ctx) {
    if (!ctx) return fail(LBP_E_INVALID, "ctx is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return LBP_OK;
}

void lbp_ctx_destroy(lbp_ctx *ctx) {
    if (!ctx) return;
    if (ctx->capture) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamDestroy(ctx->capture);
    }
    delete ctx;
}

int lbp_ctx_use_graphs(lbp_ctx *ctx, int enable) {
    if (!ctx) return fail(LBP_E_INVALID, "ctx is NULL");
    ctx->use_graphs = enable != 0;
    return LBP_OK;
}

int lbp_graph_upload(lbp_ctx *ctx, const lbp_graph_desc *desc, lbp_graph **out) {
    if (!ctx || !out) return fail(LBP_E_INVALID, "ctx or out is NULL");
    lbp_graph *g = nullptr;
    try {
        HostLayout L;
        std::string err;
        int rc = compile_desc(desc, &L, &err);
        if (rc == LBP_OK) rc = check_layout(L, &err);
        if (rc != LBP_OK) return fail(rc, err);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");

        // ---- one device allocation, carved into 256-byte aligned pieces
        struct Piece {
            const void *src;
            size_t bytes;
            size_t off;
        };
        std::vector<Piece> pcs;
        size_t total = 0;
        auto add = [&](const void *src, size_t bytes) {
            pcs.push_back(Piece{src, bytes, total});
            total += align256(std::max<size_t>(bytes, 4));
            return pcs.size() - 1;
        };
        const size_t i_m = add(nullptr, sizeof(float) * L.M);
        const size_t i_B = add(nullptr, sizeof(float) * L.VB);
        const size_t i_th = add(L.theta_panel.data(), sizeof(float) * L.VB);
        const size_t i_phi = add(L.phi_panel.data(), sizeof(float) * L.P);
        const size_t i_ft = add(L.ftile.data(), sizeof(FTile) * L.ftile.size());
        const size_t i_fvb = add(L.fvb.data(), sizeof(int32_t) * L.fvb.size());
        const size_t i_vt = add(L.vtile.data(), sizeof(VTile) * L.vtile.size());
        const size_t i_ve = add(L.vedge.data(), sizeof(int32_t) * L.vedge.size());
        const size_t i_vns = add(L.vns.data(), sizeof(int32_t) * L.vns.size());
        const size_t i_hv = add(L.hvar.data(), sizeof(HVar) * L.hvar.size());
        const size_t i_he = add(L.hedge.data(), sizeof(int32_t) * L.hedge.size());
        const size_t i_gc = add(L.gcls.data(), sizeof(GenClass) * L.gcls.size());
        const size_t i_gr = add(L.grows.data(), L.grows.size());
        const size_t i_em = add(L.edge_maddr.data(), sizeof(int32_t) * L.edge_maddr.size());
        const size_t i_es = add(L.es_off.data(), sizeof(int64_t) * L.es_off.size());
        const size_t i_vs = add(L.vs_off.data(), sizeof(int64_t) * L.vs_off.size());
        const size_t i_vn = add(L.vn.data(), sizeof(int32_t) * L.vn.size());
        const size_t i_fp = add(L.fac_phi.data(), sizeof(int32_t) * L.fac_phi.size());
        const size_t i_lp = add(L.lp_off.data(), sizeof(int64_t) * L.lp_off.size());
        const size_t i_fl = add(nullptr, sizeof(int32_t) * 4);
        const size_t i_dg = add(nullptr, sizeof(DevGraph));
        const size_t i_q = add(nullptr, sizeof(float) * L.VS);
        const size_t i_map = add(nullptr, sizeof(int32_t) * L.V);
        // work items
        std::vector<std::vector<WorkItem>> items;
        std::vector<size_t> item_piece;
        VarWork vw;
        {
            std::vector<WorkItem> mids, highs;
            add_var_work(vw, 0, L.vgroups, L.mids, L.highs, &mids, &highs);
            finish_var_work(vw, mids, highs);
        }
        for (auto &w : vw.items) items.push_back(w);
        for (const FGroup &fg : L.fgroups) {
            std::vector<WorkItem> w;
            for (int32_t t : fg.tiles) w.push_back(WorkItem{0, t});
            items.push_back(std::move(w));
        }
        for (auto &w : items) item_piece.push_back(add(w.data(), sizeof(WorkItem) * w.size()));

        g = new lbp_graph;
        g->ctx = ctx;
        e = hipMalloc((void **)&g->dmem, total);
        if (e != hipSuccess) {
            delete g;
            (void)hipGetLastError();
            return fail(LBP_E_OOM, "device allocation of " + std::to_string(total) + " bytes failed");
        }
        g->dbytes = total;
        auto ptr = [&](size_t i) { return (void *)(g->dmem + pcs[i].off); };
        hipStream_t st = ctx->stream;
        for (const Piece &p : pcs)
            if (p.src && p.bytes) {
                e = hipMemcpyAsync(g->dmem + p.off, p.src, p.bytes, hipMemcpyHostToDevice, st);
                if (e != hipSuccess) break;
            }
        if (e == hipSuccess) e = hipMemsetAsync(ptr(i_m), 0, sizeof(float) * L.M, st);
        if (e == hipSuccess) e = hipMemsetAsync(ptr(i_B), 0, sizeof(float) * L.VB, st);
        if (e == hipSuccess) e = hipMemsetAsync(ptr(i_fl), 0, sizeof(int32_t) * 4, st);

        DevGraph &h = g->host;
        h.m = (float *)ptr(i_m);
        h.mo = h.m;
        h.B = (float *)ptr(i_B);
        h.theta = (float *)ptr(i_th);
        h.phi = (float *)ptr(i_phi);
        h.ftile = (const FTile *)ptr(i_ft);
        h.fvb = (const int32_t *)ptr(i_fvb);
        h.vtile = (const VTile *)ptr(i_vt);
        h.vedge = (const int32_t *)ptr(i_ve);
        h.vns = (const int32_t *)ptr(i_vns);
        h.hvar = (const HVar *)ptr(i_hv);
        h.hedge = (const int32_t *)ptr(i_he);
        h.gcls = (const GenClass *)ptr(i_gc);
        h.grows = (const uint8_t *)ptr(i_gr);
        h.edge_maddr = (const int32_t *)ptr(i_em);
        h.es_off = (const int64_t *)ptr(i_es);
        h.vs_off = (const int64_t *)ptr(i_vs);
        h.vn = (const int32_t *)ptr(i_vn);
        h.fac_phi = (const int32_t *)ptr(i_fp);
        h.lp_off = (const int64_t *)ptr(i_lp);
        h.flag = (int32_t *)ptr(i_fl);
        h.V = (int32_t)L.V;
        h.E = (int32_t)L.E;
        h.F = (int32_t)L.F;
        h.zero_addr = L.zero_addr;
        g->dgraph = (DevGraph *)ptr(i_dg);
        g->q_tmp = (float *)ptr(i_q);
        g->map_tmp = (int32_t *)ptr(i_map);
        if (e == hipSuccess) e = hipMemcpyAsync(g->dgraph, &h, sizeof(DevGraph), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipFree(g->dmem);
            delete g;
            return hip_fail(e, "graph upload");
        }
        size_t ip = 0;
        for (size_t i = 0; i < vw.buckets.size(); ++i, ++ip) {
            Launch Lv{-1, vw.buckets[i], 0, 0, (WorkItem *)ptr(item_piece[ip])};
            Lv.n_mid = i == 0 ? vw.n_mid : 0;
            Lv.n_high = i == 0 ? vw.n_high : 0;
            Lv.n = (int32_t)vw.items[i].size() - Lv.n_mid - Lv.n_high;
            g->vl.push_back(Lv);
        }
        for (const FGroup &fg : L.fgroups) {
            g->fl.push_back(Launch{fg.kind, fg.a, fg.b, (int32_t)fg.tiles.size(), (WorkItem *)ptr(item_piece[ip])});
            ++ip;
        }
        g->fgroups = L.fgroups;
        for (const FGroup &fg : L.fgroups)
            if (fg.kind == TK_LOGL || fg.kind == TK_LOGW) g->has_logical = true;
        g->vgroups = L.vgroups;
        g->mids = L.mids;
        g->highs = L.highs;
        g->V = L.V; g->VS = L.VS; g->F = L.F; g->E = L.E; g->ES = L.ES; g->Tn = L.Tn;
        g->M = L.M; g->VB = L.VB; g->P = L.P;
        g->nvt = (int32_t)L.vtile.size();
        *out = g;
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        if (g) {
            if (g->dmem) (void)hipFree(g->dmem);
            delete g;
        }
        return fail(LBP_E_OOM, "host allocation failed");
    }
}

void lbp_graph_free(lbp_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    destroy_loops(g->loops);
    if (g->adj.dmem) (void)hipFree(g->adj.dmem);
    (void)hipFree(g->dmem);
    delete g;
}

int lbp_graph_sizes(const lbp_graph *g, int64_t out[8]) {
    if (!g || !out) return fail(LBP_E_INVALID, "graph or out is NULL");
    out[0] = g->V; out[1] = g->VS; out[2] = g->F; out[3] = g->E; out[4] = g->ES; out[5] = g->Tn;
    out[6] = (int64_t)g->dbytes;
    out[7] = g->M;
    return LBP_OK;
}

static int copy_in(lbp_graph *g, const float *values, int on_device, int64_t count, bool check_finite,
                   hipError_t (*launch)(const DevGraph *, int, const float *, hipStream_t), int n_items) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    if (count > 0 && !values) return fail(LBP_E_INVALID, "values is NULL");
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    if (count == 0) return LBP_OK;
    if (on_device) {
        HIP_TRY(launch(g->dgraph, n_items, values, st));
        return LBP_OK;
    }
    if (check_finite)
        for (int64_t i = 0; i < count; ++i)
            if (!std::isfinite(values[i])) return fail(LBP_E_INVALID, "non-finite value at " + std::to_string(i));
    float *tmp = nullptr;
    hipError_t e = hipMalloc((void **)&tmp, sizeof(float) * count);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBP_E_OOM, "staging allocation failed");
    }
    e = hipMemcpyAsync(tmp, values, sizeof(float) * count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch(g->dgraph, n_items, tmp, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "copy-in");
    return LBP_OK;
}

int lbp_set_evidence(lbp_graph *g, const float *values, int on_device) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    ++g->version;
    return copy_in(g, values, on_device, g->VS, true, launch_evidence_in, (int)g->V);
}

int lbp_set_log_potentials(lbp_graph *g, const float *values, int on_device) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    ++g->version;
    return copy_in(g, values, on_device, g->Tn, true, launch_logpot_in, (int)g->F);
}

int lbp_set_messages(lbp_graph *g, const float *values, int on_device) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    ++g->version;
    return copy_in(g, values, on_device, g->ES, true, launch_msgs_in, (int)g->E);
}

int lbp_get_messages(lbp_graph *g, float *out, int on_device) {
    if (!g || (!out && g->ES > 0)) return fail(LBP_E_INVALID, "graph or out is NULL");
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    if (g->ES == 0) return LBP_OK;
    if (on_device) {
        HIP_TRY(launch_msgs_out(g->dgraph, (int)g->E, out, st));
        return LBP_OK;
    }
    float *tmp = nullptr;
    hipError_t e = hipMalloc((void **)&tmp, sizeof(float) * g->ES);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBP_E_OOM, "staging allocation failed");
    }
    e = launch_msgs_out(g->dgraph, (int)g->E, tmp, st);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, sizeof(float) * g->ES, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "get_messages");
    return LBP_OK;
}

int lbp_reset_messages(lbp_graph *g) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    ++g->version;
    HIP_TRY(hipSetDevice(g->ctx->device));
    HIP_TRY(hipMemsetAsync(g->host.m, 0, sizeof(float) * g->M, g->ctx->stream));
    return LBP_OK;
}

int lbp_run_bp(lbp_graph *g, int32_t iters, float damping, float temperature) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    std::string why;
    if (!valid_params(iters, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    HIP_TRY(hipSetDevice(g->ctx->device));
    ++g->version;
    hipError_t e = run_loop(g->ctx, g->loops, g->dgraph, g->vl, g->fl, iters, damping, temperature);
    if (e != hipSuccess) return hip_fail(e, "iteration launch");
    g->last_T = temperature;
    return LBP_OK;
}

static int readout(lbp_graph *g, float *q, int normalized, int32_t *map, bool on_device) {
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    const TParams P = make_params(0.5f, g->last_T);
    const bool maxp = g->last_T == 0.0f;
    hipError_t e = launch_iteration(g->dgraph, g->vl, g->fl, P, maxp, st, 1);
    if (e != hipSuccess) return hip_fail(e, "belief launch");
    float *qd = q ? (on_device ? q : g->q_tmp) : nullptr;
    int32_t *md = map ? (on_device ? map : g->map_tmp) : nullptr;
    HIP_TRY(launch_readout(g->dgraph, g->nvt, maxp, P, qd, normalized, md, st));
    if (on_device) return LBP_OK;
    if (q) HIP_TRY(hipMemcpyAsync(q, g->q_tmp, sizeof(float) * g->VS, hipMemcpyDeviceToHost, st));
    if (map) HIP_TRY(hipMemcpyAsync(map, g->map_tmp, sizeof(int32_t) * g->V, hipMemcpyDeviceToHost, st));
    return lbp_graph_status(g);
}

int lbp_get_beliefs(lbp_graph *g, float *out, int normalized, int out_on_device) {
    if (!g || (!out && g->VS > 0)) return fail(LBP_E_INVALID, "graph or out is NULL");
    if (g->V == 0) return LBP_OK;
    return readout(g, out, normalized, nullptr, out_on_device != 0);
}

int lbp_decode_map(lbp_graph *g, int32_t *out, int out_on_device) {
    if (!g || (!out && g->V > 0)) return fail(LBP_E_INVALID, "graph or out is NULL");
    if (g->V == 0) return LBP_OK;
    return readout(g, nullptr, 1, out, out_on_device != 0);
}

int lbp_graph_status(lbp_graph *g) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    HIP_TRY(hipSetDevice(g->ctx->device));
    int32_t flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, g->host.flag, sizeof(int32_t), hipMemcpyDeviceToHost, g->ctx->stream));
    HIP_TRY(hipStreamSynchronize(g->ctx->stream));
    if (flag) {
        HIP_TRY(hipMemsetAsync(g->host.flag, 0, sizeof(int32_t), g->ctx->stream));
        HIP_TRY(hipStreamSynchronize(g->ctx->stream));
        return fail(LBP_E_NONFINITE, "beliefs contain NaN or infinity");
    }
    return LBP_OK;
}

int lbp_time_phase(lbp_graph *g, int32_t phase, int32_t reps, float damping, float temperature, float *ms_out) {
    if (!g || !ms_out) return fail(LBP_E_INVALID, "graph or ms_out is NULL");
    if (phase < 0 || phase > 2 || reps < 1) return fail(LBP_E_INVALID, "phase must be 0..2 and reps >= 1");
    std::string why;
    if (!valid_params(0, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    const TParams P = make_params(damping, temperature);
    const bool maxp = temperature == 0.0f;
    const int phases = phase == 0 ? 1 : phase == 1 ? 2 : 3;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    e = hipEventRecord(a, st);
    if (phases & 2) ++g->version;
    for (int32_t r = 0; r < reps && e == hipSuccess; ++r) e = launch_iteration(g->dgraph, g->vl, g->fl, P, maxp, st, phases);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "timing");
    *ms_out = ms / (float)reps;
    return LBP_OK;
}

// ---------------------------------------------------------------- adjoint
// Forward run that keeps the checkpoints the reverse sweep needs: m_t for
// t = 0, k, 2k, ... (the start of each segment of k iterations).
int lbp_run_bp_record(lbp_graph *g, int32_t iters, float damping, float temperature, int32_t ckpt_every) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    std::string why;
    if (!valid_params(iters, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    if (!(temperature > 0.0f)) return fail(LBP_E_INVALID, "the adjoint needs temperature > 0 (sum-product)");
    if (ckpt_every < 1) return fail(LBP_E_INVALID, "ckpt_every must be >= 1");
    if (g->has_logical) return fail(LBP_E_UNSUPPORTED, "the adjoint supports enumeration factors only");
    try {
        HIP_TRY(hipSetDevice(g->ctx->device));
        hipStream_t st = g->ctx->stream;
        auto &J = g->adj;
        J.valid = false;
        const int32_t k = std::min<int32_t>(ckpt_every, std::max<int32_t>(iters, 1));
        const int32_t nseg = (iters + k - 1) / k;
        const size_t M = (size_t)g->M, VB = (size_t)g->VB, P = (size_t)g->P;
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off += align256(std::max<size_t>(bytes, 4));
            return o;
        };
        const size_t o_ck = take(sizeof(float) * M * std::max(nseg, 1));
        const size_t o_seg = take(sizeof(float) * M * k);
        const size_t o_A = take(sizeof(float) * M), o_nb = take(sizeof(float) * M);
        const size_t o_Bb = take(sizeof(float) * VB), o_Bt = take(sizeof(float) * VB);
        const size_t o_z = take(sizeof(float) * VB), o_tb = take(sizeof(float) * VB);
        const size_t o_pb = take(sizeof(float) * P);
        const size_t o_v = take(sizeof(DevGraph) * (k + 2));
        if (off > J.bytes) {
            HIP_TRY(hipStreamSynchronize(st));
            if (J.dmem) (void)hipFree(J.dmem);
            J.dmem = nullptr;
            J.bytes = 0;
            hipError_t e = hipMalloc((void **)&J.dmem, off);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(LBP_E_OOM, "adjoint workspace of " + std::to_string(off) + " bytes");
            }
            J.bytes = off;
        }
        J.ckpt = (float *)(J.dmem + o_ck);
        J.seg = (float *)(J.dmem + o_seg);
        J.A = (float *)(J.dmem + o_A);
        J.nbar = (float *)(J.dmem + o_nb);
        J.Bbar = (float *)(J.dmem + o_Bb);
        J.Bt = (float *)(J.dmem + o_Bt);
        J.zeros = (float *)(J.dmem + o_z);
        J.thetabar = (float *)(J.dmem + o_tb);
        J.phibar = (float *)(J.dmem + o_pb);
        J.views = (DevGraph *)(J.dmem + o_v);
        // zero panels of the iterate buffers and of nbar must read as zero
        HIP_TRY(hipMemsetAsync(J.seg, 0, sizeof(float) * M * k, st));
        HIP_TRY(hipMemsetAsync(J.nbar, 0, sizeof(float) * M, st));
        HIP_TRY(hipMemsetAsync(J.zeros, 0, sizeof(float) * VB, st));
        std::vector<DevGraph> views(k + 2, g->host);
        for (int32_t j = 0; j < k; ++j) {
            views[j].m = J.seg + M * j;
            views[j].mo = J.seg + M * std::min(j + 1, k - 1);
            views[j].B = J.Bt;
        }
        views[k].B = J.Bt;
        views[k + 1].m = J.nbar;
        views[k + 1].mo = J.nbar;
        views[k + 1].theta = J.zeros;
        views[k + 1].B = J.Bbar;
        HIP_TRY(hipMemcpyAsync(J.views, views.data(), sizeof(DevGraph) * (k + 2), hipMemcpyHostToDevice, st));
        // the forward run, checkpointing each segment's first iterate
        ++g->version;
        for (int32_t sidx = 0; sidx < nseg; ++sidx) {
            HIP_TRY(hipMemcpyAsync(J.ckpt + M * sidx, g->host.m, sizeof(float) * M, hipMemcpyDeviceToDevice, st));
            const int32_t len = std::min(k, iters - sidx * k);
            hipError_t e = run_loop(g->ctx, g->loops, g->dgraph, g->vl, g->fl, len, damping, temperature);
            if (e != hipSuccess) return hip_fail(e, "recorded iteration launch");
        }
        HIP_TRY(hipStreamSynchronize(st));  // the host staging of the views must outlive its copy
        g->last_T = temperature;
        J.valid = true;
        J.version = g->version;
        J.iters = iters;
        J.k = k;
        J.nseg = nseg;
        J.d = damping;
        J.T = temperature;
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        return fail(LBP_E_OOM, "host allocation failed");
    }
}

int lbp_run_bp_backward(lbp_graph *g, const float *grad_q, float *grad_logpot, float *grad_evidence) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    if ((g->VS > 0 && !grad_q) || (g->Tn > 0 && !grad_logpot))
        return fail(LBP_E_INVALID, "grad_q or grad_logpot is NULL");
    auto &J = g->adj;
    if (!J.valid || J.version != g->version)
        return fail(LBP_E_STATE, "no lbp_run_bp_record since the graph's messages or inputs last changed");
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
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
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return LBP_OK;
}

// ---------------------------------------------------------------- batches
int lbp_batch_create(lbp_ctx *ctx, lbp_graph *const *graphs, int32_t num_graphs, lbp_batch **out) {
    if (!ctx || !out || (num_graphs > 0 && !graphs) || num_graphs < 0)
        return fail(LBP_E_INVALID, "bad batch arguments");
    for (int32_t i = 0; i < num_graphs; ++i)
        if (!graphs[i] || graphs[i]->ctx->device != ctx->device)
            return fail(LBP_E_INVALID, "graph " + std::to_string(i) + " is NULL or on another device");
    lbp_batch *b = nullptr;
    try {
        HIP_TRY(hipSetDevice(ctx->device));
        // merge launches by shape: belief-low by bucket, belief-high, factor kernels by (kind, a, b)
        struct Key {
            int32_t kind, a, b;
            bool operator==(const Key &o) const { return kind == o.kind && a == o.a && b == o.b; }
        };
        std::vector<Key> fkeys;
        std::vector<std::vector<WorkItem>> fitems;
        VarWork vw;
        std::vector<WorkItem> mids, highs;
        auto slot = [](std::vector<Key> &keys, std::vector<std::vector<WorkItem>> &its, Key k) -> std::vector<WorkItem> & {
            for (size_t i = 0; i < keys.size(); ++i)
                if (keys[i] == k) return its[i];
            keys.push_back(k);
            its.emplace_back();
            return its.back();
        };
        for (int32_t gi = 0; gi < num_graphs; ++gi) {
            const lbp_graph *g = graphs[gi];
            // the graph's item lists are on the device; rebuild them from its groups
            add_var_work(vw, gi, g->vgroups, g->mids, g->highs, &mids, &highs);
            for (const FGroup &fg : g->fgroups) {
                auto &v = slot(fkeys, fitems, Key{fg.kind, fg.a, fg.b});
                for (int32_t t : fg.tiles) v.push_back(WorkItem{gi, t});
            }
        }
        finish_var_work(vw, mids, highs);
        std::vector<std::vector<WorkItem>> &vitems = vw.items;
        size_t total = align256(sizeof(DevGraph) * std::max(1, num_graphs));
        std::vector<size_t> voff, foff;
        for (auto &v : vitems) {
            voff.push_back(total);
            total += align256(sizeof(WorkItem) * std::max<size_t>(1, v.size()));
        }
        for (auto &v : fitems) {
            foff.push_back(total);
            total += align256(sizeof(WorkItem) * std::max<size_t>(1, v.size()));
        }
        b = new lbp_batch;
        b->ctx = ctx;
        b->graphs.assign(graphs, graphs + num_graphs);
        hipError_t e = hipMalloc((void **)&b->dmem, total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return fail(LBP_E_OOM, "batch allocation failed");
        }
        std::vector<DevGraph> hg;
        for (int32_t gi = 0; gi < num_graphs; ++gi) hg.push_back(graphs[gi]->host);
        b->dgraphs = (DevGraph *)b->dmem;
        hipStream_t st = ctx->stream;
        if (num_graphs) e = hipMemcpyAsync(b->dgraphs, hg.data(), sizeof(DevGraph) * num_graphs, hipMemcpyHostToDevice, st);
        for (size_t i = 0; i < vitems.size() && e == hipSuccess; ++i) {
            e = hipMemcpyAsync(b->dmem + voff[i], vitems[i].data(), sizeof(WorkItem) * vitems[i].size(),
                               hipMemcpyHostToDevice, st);
            Launch Lv{-1, vw.buckets[i], 0, 0, (WorkItem *)(b->dmem + voff[i])};
            Lv.n_mid = i == 0 ? vw.n_mid : 0;
            Lv.n_high = i == 0 ? vw.n_high : 0;
            Lv.n = (int32_t)vitems[i].size() - Lv.n_mid - Lv.n_high;
            b->vl.push_back(Lv);
        }
        for (size_t i = 0; i < fitems.size() && e == hipSuccess; ++i) {
            e = hipMemcpyAsync(b->dmem + foff[i], fitems[i].data(), sizeof(WorkItem) * fitems[i].size(),
                               hipMemcpyHostToDevice, st);
            b->fl.push_back(Launch{fkeys[i].kind, fkeys[i].a, fkeys[i].b, (int32_t)fitems[i].size(),
                                   (WorkItem *)(b->dmem + foff[i])});
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipFree(b->dmem);
            delete b;
            return hip_fail(e, "batch upload");
        }
        *out = b;
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        if (b) {
            if (b->dmem) (void)hipFree(b->dmem);
            delete b;
        }
        return fail(LBP_E_OOM, "host allocation failed");
    }
}

int lbp_batch_run(lbp_batch *b, int32_t iters, float damping, float temperature) {
    if (!b) return fail(LBP_E_INVALID, "batch is NULL");
    std::string why;
    if (!valid_params(iters, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    HIP_TRY(hipSetDevice(b->ctx->device));
    hipError_t e = run_loop(b->ctx, b->loops, b->dgraphs, b->vl, b->fl, iters, damping, temperature);
    if (e != hipSuccess) return hip_fail(e, "batch iteration launch");
    for (lbp_graph *g : b->graphs) {
        g->last_T = temperature;
        ++g->version;
    }
    return LBP_OK;
}

void lbp_batch_free(lbp_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    destroy_loops(b->loops);
    (void)hipFree(b->dmem);
    delete b;
}

}  // extern "C"
