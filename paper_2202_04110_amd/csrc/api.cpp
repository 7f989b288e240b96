// C-ABI of liblbp.so (declared in include/lbp.h): contexts, graph upload,
// iteration driver, read-out, state exchange and batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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
    int32_t kind;  // -1 belief-low, -2 belief-high, TK_* factor kernels
    int32_t a, b;  // belief-low: bucket; PAIR: states; LOGW: chunk bucket
    int32_t n;
    WorkItem *items;  // device
};

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
            e = L.kind == -1 ? launch_belief_low(gs, L.items, L.n, L.a, st) : launch_belief_high(gs, L.items, L.n, st);
            if (e != hipSuccess) return e;
        }
    if (phases & 2)
        for (const Launch &L : fl) {
            switch (L.kind) {
            case TK_PAIR: e = launch_pair(gs, L.items, L.n, L.a, L.b, maxp, P, st); break;
            case TK_LOGL: e = launch_logl(gs, L.items, L.n, maxp, P, st); break;
            case TK_LOGW: e = launch_logw(gs, L.items, L.n, L.a, maxp, P, st); break;
            default: e = launch_gen(gs, L.items, L.n, maxp, P, st); break;
            }
            if (e != hipSuccess) return e;
        }
    return e;
}

}  // namespace

struct lbp_ctx {
    int device;
    hipStream_t stream;
};

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
    std::vector<int32_t> ftile_count_by_group, hvar_count;
    int32_t nhvar = 0;
    float last_T = 0.0f;
};

struct lbp_batch {
    lbp_ctx *ctx = nullptr;
    std::vector<lbp_graph *> graphs;
    char *dmem = nullptr;
    DevGraph *dgraphs = nullptr;
    std::vector<Launch> vl, fl;
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

void lbp_ctx_destroy(lbp_ctx *ctx) { delete ctx; }

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
        for (const VGroup &vg : L.vgroups) {
            std::vector<WorkItem> w;
            for (int32_t t : vg.tiles) w.push_back(WorkItem{0, t});
            items.push_back(std::move(w));
        }
        {
            std::vector<WorkItem> w;
            for (size_t i = 0; i < L.hvar.size(); ++i) w.push_back(WorkItem{0, (int32_t)i});
            items.push_back(std::move(w));
        }
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
        for (const VGroup &vg : L.vgroups) {
            g->vl.push_back(Launch{-1, vg.bucket, 0, (int32_t)vg.tiles.size(), (WorkItem *)ptr(item_piece[ip])});
            ++ip;
        }
        if (!L.hvar.empty()) g->vl.push_back(Launch{-2, 0, 0, (int32_t)L.hvar.size(), (WorkItem *)ptr(item_piece[ip])});
        ++ip;
        for (const FGroup &fg : L.fgroups) {
            g->fl.push_back(Launch{fg.kind, fg.a, fg.b, (int32_t)fg.tiles.size(), (WorkItem *)ptr(item_piece[ip])});
            ++ip;
        }
        g->fgroups = L.fgroups;
        g->vgroups = L.vgroups;
        g->nhvar = (int32_t)L.hvar.size();
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
    return copy_in(g, values, on_device, g->VS, true, launch_evidence_in, (int)g->V);
}

int lbp_set_log_potentials(lbp_graph *g, const float *values, int on_device) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    return copy_in(g, values, on_device, g->Tn, true, launch_logpot_in, (int)g->F);
}

int lbp_set_messages(lbp_graph *g, const float *values, int on_device) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
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
    HIP_TRY(hipSetDevice(g->ctx->device));
    HIP_TRY(hipMemsetAsync(g->host.m, 0, sizeof(float) * g->M, g->ctx->stream));
    return LBP_OK;
}

int lbp_run_bp(lbp_graph *g, int32_t iters, float damping, float temperature) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    std::string why;
    if (!valid_params(iters, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    HIP_TRY(hipSetDevice(g->ctx->device));
    const TParams P = make_params(damping, temperature);
    const bool maxp = temperature == 0.0f;
    for (int32_t it = 0; it < iters; ++it) {
        hipError_t e = launch_iteration(g->dgraph, g->vl, g->fl, P, maxp, g->ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "iteration launch");
    }
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
        std::vector<Key> vkeys, fkeys;
        std::vector<std::vector<WorkItem>> vitems, fitems;
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
            for (const VGroup &vg : g->vgroups) {
                auto &v = slot(vkeys, vitems, Key{-1, vg.bucket, 0});
                for (int32_t t : vg.tiles) v.push_back(WorkItem{gi, t});
            }
            if (g->nhvar) {
                auto &v = slot(vkeys, vitems, Key{-2, 0, 0});
                for (int32_t t = 0; t < g->nhvar; ++t) v.push_back(WorkItem{gi, t});
            }
            for (const FGroup &fg : g->fgroups) {
                auto &v = slot(fkeys, fitems, Key{fg.kind, fg.a, fg.b});
                for (int32_t t : fg.tiles) v.push_back(WorkItem{gi, t});
            }
        }
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
            b->vl.push_back(Launch{vkeys[i].kind, vkeys[i].a, 0, (int32_t)vitems[i].size(), (WorkItem *)(b->dmem + voff[i])});
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
    const TParams P = make_params(damping, temperature);
    const bool maxp = temperature == 0.0f;
    for (int32_t it = 0; it < iters; ++it) {
        hipError_t e = launch_iteration(b->dgraphs, b->vl, b->fl, P, maxp, b->ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "batch iteration launch");
    }
    for (lbp_graph *g : b->graphs) g->last_T = temperature;
    return LBP_OK;
}

void lbp_batch_free(lbp_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    (void)hipFree(b->dmem);
    delete b;
}

}  // extern "C"
