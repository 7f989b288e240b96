// C-ABI of liblbp.so (declared in include/lbp.h): contexts, graph upload,
// iteration driver, read-out, state exchange, the reverse sweep and batches.
// The work itself lives in runtime.cpp and kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "runtime.h"

using namespace lbp;

namespace {

int fail(int code, const std::string &msg) { return set_error(code, msg); }

int copy_in(lbp_graph *g, const float *values, int on_device, int64_t count,
            hipError_t (*launch)(const DevGraph *, int, const float *, hipStream_t), int n_items) {
    if (count > 0 && !values) return fail(LBP_E_INVALID, "values is NULL");
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    if (count == 0) return LBP_OK;
    if (on_device) {
        HIP_TRY(launch(g->dgraph, n_items, values, st));
        return LBP_OK;
    }
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
    if (e != hipSuccess) return hip_error(e, "copy-in");
    return LBP_OK;
}

}  // namespace

extern "C" {

const char *lbp_last_error(void) { return last_error(); }

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
    if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(LBP_E_INVALID, "device index out of range");
    HIP_TRY(hipSetDevice(device));
    // set-up of the fixed scratch of lbp_run_bp_until_noalloc on this device
    float *scratch_addr = nullptr;
    e = noalloc_scratch_address(device, &scratch_addr);
    if (e != hipSuccess) return hip_error(e, "scratch address lookup");
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

int lbp_ctx_use_graphs(lbp_ctx *ctx, int enable) {
    if (!ctx) return fail(LBP_E_INVALID, "ctx is NULL");
    ctx->use_graphs = enable != 0;
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

int lbp_graph_upload(lbp_ctx *ctx, const lbp_graph_desc *desc, lbp_graph **out) {
    if (!ctx || !out) return fail(LBP_E_INVALID, "ctx or out is NULL");
    try {
        HostLayout L;
        std::string err;
        int rc = compile_desc(desc, &L, &err);
        if (rc == LBP_OK) rc = check_layout(L, &err);
        if (rc != LBP_OK) return fail(rc, err);
        HIP_TRY(hipSetDevice(ctx->device));
        return graph_create(ctx, L, true, nullptr, ctx->stream, out);
    } catch (const std::bad_alloc &) {
        return fail(LBP_E_OOM, "host allocation failed");
    }
}

void lbp_graph_free(lbp_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    graph_destroy(g);
}

int lbp_graph_sizes(const lbp_graph *g, int64_t out[8]) {
    if (!g || !out) return fail(LBP_E_INVALID, "graph or out is NULL");
    out[0] = g->V; out[1] = g->VS; out[2] = g->F; out[3] = g->E; out[4] = g->ES; out[5] = g->Tn;
    out[6] = (int64_t)g->dbytes;
    out[7] = g->M;
    return LBP_OK;
}

int lbp_set_evidence(lbp_graph *g, const float *values, int on_device) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    ++g->version;
    return copy_in(g, values, on_device, g->VS, launch_evidence_in, (int)g->V);
}

int lbp_set_log_potentials(lbp_graph *g, const float *values, int on_device) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    ++g->version;
    return copy_in(g, values, on_device, g->Tn, launch_logpot_in, (int)g->F);
}

int lbp_set_messages(lbp_graph *g, const float *values, int on_device) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    ++g->version;
    return copy_in(g, values, on_device, g->ES, launch_msgs_in, (int)g->E);
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
    if (e != hipSuccess) return hip_error(e, "get_messages");
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
    hipError_t e = hipErrorInvalidValue;
    if (g->use_resident) {
        e = launch_solve_resident(g->dgraph, g->plan, iters, temperature == 0.0f, make_params(damping, temperature),
                                  g->ctx->stream);
        if (e != hipSuccess) {
            // refused at launch (LDS size or configuration): launched
            // iterations from here on, for this graph
            (void)hipGetLastError();
            g->use_resident = g->resident_ok = false;
        }
    }
    if (!g->use_resident)
        e = run_loop(g->ctx, g->loops, g->dgraph, g->use_fused ? g->fused : nullptr, g->vl, g->fl, iters, damping,
                     temperature);
    if (e != hipSuccess) return hip_error(e, "iteration launch");
    g->last_T = temperature;
    return LBP_OK;
}

int lbp_graph_use_resident(lbp_graph *g, int enable) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    if (enable && !g->resident_ok) return fail(LBP_E_INVALID, "the graph does not fit the resident solver");
    g->use_resident = enable != 0;
    return LBP_OK;
}

int lbp_graph_resident_state(const lbp_graph *g, int32_t out[2]) {
    if (!g || !out) return fail(LBP_E_INVALID, "graph or out is NULL");
    out[0] = g->resident_ok;
    out[1] = g->use_resident;
    return LBP_OK;
}

int lbp_run_bp_until(lbp_graph *g, int32_t max_iters, float damping, float temperature, float tol,
                     int32_t check_every, int32_t *iters_done, float *residual_out) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    std::string why;
    if (!valid_params(max_iters, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    if (!(tol >= 0.0f) || !std::isfinite(tol)) return fail(LBP_E_INVALID, "tol must be finite and >= 0");
    if (check_every < 1) return fail(LBP_E_INVALID, "check_every must be >= 1");
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    const size_t mb = align256(sizeof(float) * std::max<int64_t>(1, g->M));
    const int nb = residual_blocks((int)g->E);
    if (!g->conv) {
        hipError_t e = hipMalloc((void **)&g->conv, mb + align256(sizeof(float) * (nb + 1)));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            g->conv = nullptr;
            return fail(LBP_E_OOM, "convergence workspace");
        }
    }
    float *mprev = (float *)g->conv, *partial = (float *)(g->conv + mb), *res = partial + nb;
    ++g->version;
    g->last_T = temperature;
    int32_t done = 0;
    float r = 0.0f;
    while (done < max_iters) {
        const int32_t c = std::min(check_every, max_iters - done);
        hipError_t e = hipSuccess;
        if (c > 1)
            e = run_loop(g->ctx, g->loops, g->dgraph, g->use_fused ? g->fused : nullptr, g->vl, g->fl, c - 1, damping,
                         temperature);
        if (e == hipSuccess) e = hipMemcpyAsync(mprev, g->host.m, sizeof(float) * g->M, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = run_loop(g->ctx, g->loops, g->dgraph, nullptr, g->vl, g->fl, 1, damping, temperature);
        if (e == hipSuccess) e = launch_residual(g->dgraph, (int)g->E, mprev, partial, res, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&r, res, sizeof(float), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_error(e, "iteration launch");
        done += c;
        if (r < tol) break;
    }
    if (iters_done) *iters_done = done;
    if (residual_out) *residual_out = r;
    return LBP_OK;
}

int lbp_bandwidth_probe(lbp_ctx *ctx, int32_t kind, const void *src, void *dst, int64_t bytes, int32_t blocks,
                        int32_t reps, float *ms_out) {
    if (!ctx || !ms_out) return fail(LBP_E_INVALID, "ctx or ms_out is NULL");
    if (kind < 0 || kind > 3) return fail(LBP_E_INVALID, "kind must be 0..3");
    if (bytes <= 0 || bytes % (kind == 3 ? 80 : 16) != 0)
        return fail(LBP_E_INVALID, "bytes must be a positive multiple of 16 (80 for kind 3)");
    if (blocks < 1 || reps < 1) return fail(LBP_E_INVALID, "blocks and reps must be >= 1");
    if ((kind != 2 && (!src || ((uintptr_t)src & 15))) || (!dst || ((uintptr_t)dst & 15)))
        return fail(LBP_E_INVALID, "src and dst must be non-NULL and 16-byte aligned");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch_stream_probe(kind, src, dst, bytes, blocks, st);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, st);
    for (int32_t r = 0; r < reps && e == hipSuccess; ++r) e = launch_stream_probe(kind, src, dst, bytes, blocks, st);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_error(e, "bandwidth probe");
    *ms_out = ms / (float)reps;
    return LBP_OK;
}

static_assert(LBP_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes, "scratch size in lbp.h and kernels.h differ");

int lbp_run_bp_until_noalloc(lbp_graph *g, int32_t max_iters, float damping, float temperature, float tol,
                             int32_t check_every, int32_t *iters_done, float *residual_out) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    std::string why;
    if (!valid_params(max_iters, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    if (!(tol >= 0.0f) || !std::isfinite(tol)) return fail(LBP_E_INVALID, "tol must be finite and >= 0");
    if (check_every < 1) return fail(LBP_E_INVALID, "check_every must be >= 1");
    const size_t mb = align256(sizeof(float) * std::max<int64_t>(1, g->M));
    const int nb = residual_blocks((int)g->E);
    const size_t need = mb + sizeof(float) * (size_t)(nb + 1);
    if (need > kNoAllocScratchBytes)
        return fail(LBP_E_UNSUPPORTED, "the graph needs " + std::to_string(need) +
                                           " bytes of scratch, more than the fixed " +
                                           std::to_string(kNoAllocScratchBytes));
    HIP_TRY(hipSetDevice(g->ctx->device));
    float *base = nullptr;
    HIP_TRY(noalloc_scratch_address(g->ctx->device, &base));
    hipStream_t st = g->ctx->stream;
    float *mprev = base, *partial = reinterpret_cast<float *>(reinterpret_cast<char *>(base) + mb),
          *res = partial + nb;
    const TParams P = make_params(damping, temperature);
    const bool maxp = temperature == 0.0f;
    ++g->version;
    g->last_T = temperature;
    int32_t done = 0;
    float r = 0.0f;
    // the kernels of lbp_run_bp_until, launched one by one (no captured
    // loop: instantiating one allocates)
    while (done < max_iters) {
        const int32_t c = std::min(check_every, max_iters - done);
        hipError_t e = hipSuccess;
        if (c > 1)
            e = launch_loop(g->dgraph, g->use_fused ? g->fused : nullptr, g->vl, g->fl, c - 1, P, maxp, st);
        if (e == hipSuccess) e = hipMemcpyAsync(mprev, g->host.m, sizeof(float) * g->M, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = launch_loop(g->dgraph, nullptr, g->vl, g->fl, 1, P, maxp, st);
        if (e == hipSuccess) e = launch_residual(g->dgraph, (int)g->E, mprev, partial, res, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&r, res, sizeof(float), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_error(e, "iteration launch");
        done += c;
        if (r < tol) break;
    }
    if (iters_done) *iters_done = done;
    if (residual_out) *residual_out = r;
    return LBP_OK;
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

static int readout(lbp_graph *g, float *q, int normalized, int32_t *map, bool on_device) {
    HIP_TRY(hipSetDevice(g->ctx->device));
    int rc = graph_readout(g, q, normalized, map, on_device, g->ctx->stream);
    if (rc != LBP_OK || on_device) return rc;
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

int lbp_time_phase(lbp_graph *g, int32_t phase, int32_t reps, float damping, float temperature, float *ms_out) {
    if (!g || !ms_out) return fail(LBP_E_INVALID, "graph or ms_out is NULL");
    if (phase < 0 || phase > 3 || reps < 1) return fail(LBP_E_INVALID, "phase must be 0..3 and reps >= 1");
    if (phase == 3 && !g->fused) return fail(LBP_E_INVALID, "the graph has no fused iteration");
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
        return hip_error(e, "hipEventCreate");
    }
    e = hipEventRecord(a, st);
    if (phases & 2) ++g->version;
    if (phase == 2 || phase == 3) {
        // iterations as lbp_run_bp runs them (phase 3: fused, in pairs)
        if (e == hipSuccess)
            e = launch_loop(g->dgraph, phase == 3 ? g->fused : nullptr, g->vl, g->fl, 2 * reps, P, maxp, st);
        reps *= 2;
    } else {
        for (int32_t r = 0; r < reps && e == hipSuccess; ++r)
            e = launch_iteration(g->dgraph, g->vl, g->fl, P, maxp, st, phases);
    }
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_error(e, "timing");
    *ms_out = ms / (float)reps;
    return LBP_OK;
}

// ---------------------------------------------------------------- autotuner
namespace {

std::vector<Launch *> all_launches(std::vector<Launch> &vl, std::vector<Launch> &fl) {
    std::vector<Launch *> v;
    for (Launch &L : vl) v.push_back(&L);
    for (Launch &L : fl) v.push_back(&L);
    return v;
}

// Times `reps` whole two-phase iterations with the groups' current shapes
// (after one warm-up iteration).
hipError_t time_iterations(const DevGraph *gs, const std::vector<Launch> &vl, const std::vector<Launch> &fl,
                           const TParams &P, bool maxp, hipStream_t st, int reps, hipEvent_t a, hipEvent_t b,
                           float *ms) {
    hipError_t e = launch_iteration(gs, vl, fl, P, maxp, st, 3);
    if (e == hipSuccess) e = hipEventRecord(a, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_iteration(gs, vl, fl, P, maxp, st, 3);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    *ms /= (float)reps;
    return e;
}

// Picks, per launch group, the shape that makes whole two-phase iterations
// fastest, the other groups at their current shapes, in two passes over the
// groups: variable phase {swizzle off, on}; lane-per-item factor kernels
// {1, 2, 4 wavefronts per block} x {swizzle off, on}; generic enumeration
// launches keep their fixed shape.  Timing whole iterations rather than one
// launch at a time sees what one phase leaves in the XCDs' L2 for the next:
// a bipartite layer's factor tiles swizzled into per-XCD runs are read by
// the column groups of the same XCD (RBM 784x500: 9.1 against 10.6 us per
// iteration unswizzled), which a launch timed alone cannot show.
int tune_launches(const DevGraph *gs, std::vector<Launch> &vl, std::vector<Launch> &fl, float d, float T, int reps,
                  hipStream_t st, float *best_ms) {
    const TParams P = make_params(d, T);
    const bool maxp = T == 0.0f;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_error(e, "hipEventCreate");
    }
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        int idx = 0;
        for (Launch *L : all_launches(vl, fl)) {
            const bool variable = L->kind == -1;
            std::vector<LaunchShape> cand;
            if (variable) {
                cand = {LaunchShape{4, 0}, LaunchShape{4, 1}};
            } else if (L->kind == TK_GEN) {
                cand = {L->shape};
            } else {
                for (int w : {1, 2, 4})
                    for (int z : {0, 1}) cand.push_back(LaunchShape{w, z});
            }
            LaunchShape best = L->shape;
            float best_t = 1e30f;
            for (const LaunchShape &c : cand) {
                L->shape = c;
                float ms = 0.0f;
                e = time_iterations(gs, vl, fl, P, maxp, st, reps, a, b, &ms);
                if (e != hipSuccess) break;
                if (ms < best_t) {
                    best_t = ms;
                    best = c;
                }
            }
            L->shape = best;
            if (best_ms) best_ms[idx] = best_t;
            ++idx;
            if (e != hipSuccess) break;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_error(e, "autotune");
    return LBP_OK;
}

// The fused launches' own shapes (waves per block x variant), then fused or
// two-phase iterations, whichever is faster: *use_fused.  gs / fused /
// stride as for launch_loop.  Moves the messages (the caller restores them).
int tune_fused(const DevGraph *gs, const DevGraph *fused, int32_t stride, const std::vector<Launch> &vl,
               std::vector<Launch> &fl, float d, float T, int reps, hipStream_t st, bool *use_fused) {
    const TParams P = make_params(d, T);
    const bool maxp = T == 0.0f;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    auto time_loop = [&](const DevGraph *fz, float *ms) {
        hipError_t x = launch_loop(gs, fz, vl, fl, 2, P, maxp, st, stride);  // warm-up
        if (x == hipSuccess) x = hipEventRecord(a, st);
        if (x == hipSuccess) x = launch_loop(gs, fz, vl, fl, 2 * reps, P, maxp, st, stride);
        if (x == hipSuccess) x = hipEventRecord(b, st);
        if (x == hipSuccess) x = hipEventSynchronize(b);
        if (x == hipSuccess) x = hipEventElapsedTime(ms, a, b);
        return x;
    };
    for (Launch &L : fl) {
        LaunchShape best = L.fshape;
        float best_t = 1e30f;
        for (int w : {1, 2, 4})
            for (int v : {0, 1, 2, 3}) {
                if (e != hipSuccess) break;
                L.fshape = LaunchShape{w, v & 1, v >> 1};
                float ms = 0.0f;
                e = time_loop(fused, &ms);
                if (e == hipSuccess && ms < best_t) {
                    best_t = ms;
                    best = L.fshape;
                }
            }
        L.fshape = best;
    }
    float t2 = 0.0f, tf = 0.0f;
    if (e == hipSuccess) e = time_loop(nullptr, &t2);
    if (e == hipSuccess) e = time_loop(fused, &tf);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_error(e, "autotune fused");
    *use_fused = tf < t2;
    return LBP_OK;
}

}  // namespace

int lbp_graph_num_launches(const lbp_graph *g, int32_t *n_out) {
    if (!g || !n_out) return fail(LBP_E_INVALID, "graph or n_out is NULL");
    *n_out = (int32_t)(g->vl.size() + g->fl.size());
    return LBP_OK;
}

int lbp_graph_get_launch(const lbp_graph *g, int32_t i, int32_t out[9]) {
    if (!g || !out) return fail(LBP_E_INVALID, "graph or out is NULL");
    const int32_t nv = (int32_t)g->vl.size(), nf = (int32_t)g->fl.size();
    if (i < 0 || i >= nv + nf) return fail(LBP_E_INVALID, "launch index out of range");
    const Launch &L = i < nv ? g->vl[i] : g->fl[i - nv];
    out[0] = i < nv ? 0 : 1;
    out[1] = L.kind;
    out[2] = L.a;
    out[3] = L.b;
    out[4] = L.shape.wpb;
    out[5] = L.shape.swizzle;
    out[6] = L.n + L.n_mid + L.n_high;
    out[7] = L.fshape.wpb;
    out[8] = L.fshape.swizzle | (L.fshape.early << 1);
    return LBP_OK;
}

int lbp_graph_set_fused_launch(lbp_graph *g, int32_t i, int32_t waves_per_block, int32_t variant) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    const int32_t nv = (int32_t)g->vl.size(), nf = (int32_t)g->fl.size();
    if (i < nv || i >= nv + nf || !g->fused) return fail(LBP_E_INVALID, "not a launch with a fused variant");
    if (variant < 0 || variant > 3 || (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4))
        return fail(LBP_E_INVALID, "waves_per_block must be 1, 2 or 4 and variant 0 to 3");
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    destroy_loops(g->loops);
    g->fl[i - nv].fshape = LaunchShape{waves_per_block, variant & 1, variant >> 1};
    return LBP_OK;
}

int lbp_graph_set_launch(lbp_graph *g, int32_t i, int32_t waves_per_block, int32_t swizzle) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    const int32_t nv = (int32_t)g->vl.size(), nf = (int32_t)g->fl.size();
    if (i < 0 || i >= nv + nf) return fail(LBP_E_INVALID, "launch index out of range");
    if (swizzle != 0 && swizzle != 1) return fail(LBP_E_INVALID, "swizzle must be 0 or 1");
    Launch &L = i < nv ? g->vl[i] : g->fl[i - nv];
    const bool fixed = i < nv || L.kind == TK_GEN;
    if (fixed ? waves_per_block != 4 : (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4))
        return fail(LBP_E_INVALID, "waves_per_block must be 1, 2 or 4 (4 for this launch)");
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    destroy_loops(g->loops);
    L.shape = LaunchShape{waves_per_block, swizzle};
    return LBP_OK;
}

int lbp_graph_use_fused(lbp_graph *g, int enable) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    if (enable && !g->fused) return fail(LBP_E_INVALID, "the graph has no fused iteration");
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    destroy_loops(g->loops);
    g->use_fused = enable != 0;
    return LBP_OK;
}

int lbp_graph_fused_state(const lbp_graph *g, int32_t out[2]) {
    if (!g || !out) return fail(LBP_E_INVALID, "graph or out is NULL");
    out[0] = g->fused != nullptr;
    out[1] = g->use_fused;
    return LBP_OK;
}

int lbp_autotune(lbp_graph *g, float damping, float temperature, int32_t reps, float *best_ms_out) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    std::string why;
    if (!valid_params(0, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    if (reps < 1) return fail(LBP_E_INVALID, "reps must be >= 1");
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    // the factor kernels update the messages: keep and restore them
    float *save = nullptr;
    hipError_t e = hipMalloc((void **)&save, sizeof(float) * g->M);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBP_E_OOM, "autotune message backup");
    }
    e = hipMemcpyAsync(save, g->host.m, sizeof(float) * g->M, hipMemcpyDeviceToDevice, st);
    int rc = e == hipSuccess ? tune_launches(g->dgraph, g->vl, g->fl, damping, temperature, reps, st, best_ms_out)
                             : hip_error(e, "autotune backup");
    if (rc == LBP_OK && g->fused)
        rc = tune_fused(g->dgraph, g->fused, 1, g->vl, g->fl, damping, temperature, reps, st, &g->use_fused);
    // loops captured before the shapes and the iteration form changed would
    // replay the old launches: drop them before timing the launched loop
    (void)hipStreamSynchronize(st);
    destroy_loops(g->loops);
    if (rc == LBP_OK && g->resident_ok) {
        // the resident solver against the launched iterations chosen above
        const TParams P = make_params(damping, temperature);
        const bool maxp = temperature == 0.0f;
        hipEvent_t a = nullptr, b = nullptr;
        float tl = 0.0f, tr = 0.0f;
        hipError_t x = hipEventCreate(&a);
        if (x == hipSuccess) x = hipEventCreate(&b);
        if (x == hipSuccess) x = launch_solve_resident(g->dgraph, g->plan, 2, maxp, P, st);  // warm-up
        if (x == hipSuccess) x = hipEventRecord(a, st);
        if (x == hipSuccess) x = launch_solve_resident(g->dgraph, g->plan, 2 * reps, maxp, P, st);
        if (x == hipSuccess) x = hipEventRecord(b, st);
        if (x == hipSuccess) x = hipEventSynchronize(b);
        if (x == hipSuccess) x = hipEventElapsedTime(&tr, a, b);
        // launched iterations as lbp_run_bp runs them: a captured loop,
        // captured on the first call and replayed on the timed one
        const DevGraph *fz = g->use_fused ? g->fused : nullptr;
        if (x == hipSuccess) x = run_loop(g->ctx, g->loops, g->dgraph, fz, g->vl, g->fl, 2 * reps, damping, temperature);
        if (x == hipSuccess) x = hipEventRecord(a, st);
        if (x == hipSuccess) x = run_loop(g->ctx, g->loops, g->dgraph, fz, g->vl, g->fl, 2 * reps, damping, temperature);
        if (x == hipSuccess) x = hipEventRecord(b, st);
        if (x == hipSuccess) x = hipEventSynchronize(b);
        if (x == hipSuccess) x = hipEventElapsedTime(&tl, a, b);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (x == hipSuccess) {
            g->use_resident = tr < tl;
        } else {
            // the resident solver was refused (LDS size or configuration)
            (void)hipGetLastError();
            (void)hipStreamSynchronize(st);
            g->use_resident = g->resident_ok = false;
        }
    }
    e = hipMemcpyAsync(g->host.m, save, sizeof(float) * g->M, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(save);
    destroy_loops(g->loops);
    if (rc != LBP_OK) return rc;
    if (e != hipSuccess) return hip_error(e, "autotune restore");
    return LBP_OK;
}

// ---------------------------------------------------------------- adjoint
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
        int rc = adjoint_prepare(g, iters, damping, temperature, ckpt_every, nullptr, st);
        if (rc != LBP_OK) return rc;
        ++g->version;
        const int32_t k = g->adj.k;
        for (int32_t sidx = 0; sidx < g->adj.nseg; ++sidx) {
            rc = adjoint_checkpoint(g, sidx, st);
            if (rc != LBP_OK) return rc;
            const int32_t len = std::min(k, iters - sidx * k);
            hipError_t e = run_loop(g->ctx, g->loops, g->dgraph, g->use_fused ? g->fused : nullptr, g->vl, g->fl, len,
                                    damping, temperature);
            if (e != hipSuccess) return hip_error(e, "recorded iteration launch");
        }
        g->last_T = temperature;
        adjoint_finish_record(g);
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        return fail(LBP_E_OOM, "host allocation failed");
    }
}

int lbp_run_bp_backward(lbp_graph *g, const float *grad_q, float *grad_logpot, float *grad_evidence) {
    if (!g) return fail(LBP_E_INVALID, "graph is NULL");
    if ((g->VS > 0 && !grad_q) || (g->Tn > 0 && !grad_logpot))
        return fail(LBP_E_INVALID, "grad_q or grad_logpot is NULL");
    if (!g->adj.valid || g->adj.version != g->version)
        return fail(LBP_E_STATE, "no lbp_run_bp_record since the graph's messages or inputs last changed");
    HIP_TRY(hipSetDevice(g->ctx->device));
    return adjoint_backward(g, grad_q, grad_logpot, grad_evidence, g->ctx->stream);
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
        LaunchLists ll;
        std::vector<WorkItem> mids, highs, cols;
        for (int32_t gi = 0; gi < num_graphs; ++gi) add_to_lists(ll, gi, graphs[gi]->shape, &mids, &highs, &cols);
        finish_lists(ll, mids, highs, cols, true);
        const size_t gbytes = align256(sizeof(DevGraph) * 3 * std::max(1, num_graphs));
        const size_t total = gbytes + lists_bytes(ll);
        b = new lbp_batch;
        b->ctx = ctx;
        b->graphs.assign(graphs, graphs + num_graphs);
        hipError_t e = hipMalloc((void **)&b->dmem, total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return fail(LBP_E_OOM, "batch allocation failed");
        }
        // descriptors, then (when every graph has a fused form) each graph's
        // m -> m2 view and then each graph's m2 -> m view
        std::vector<DevGraph> hg;
        for (int32_t gi = 0; gi < num_graphs; ++gi) hg.push_back(graphs[gi]->host);
        bool fusable = num_graphs > 0;
        for (int32_t gi = 0; gi < num_graphs; ++gi) fusable = fusable && graphs[gi]->m2;
        if (fusable) {
            for (int32_t gi = 0; gi < num_graphs; ++gi) {
                hg.push_back(graphs[gi]->host);
                hg.back().mo = graphs[gi]->m2;
            }
            for (int32_t gi = 0; gi < num_graphs; ++gi) {
                hg.push_back(graphs[gi]->host);
                hg.back().m = graphs[gi]->m2;
                hg.back().mo = graphs[gi]->host.m;
            }
        }
        b->dgraphs = (DevGraph *)b->dmem;
        b->fviews = fusable ? b->dgraphs + num_graphs : nullptr;
        hipStream_t st = ctx->stream;
        if (num_graphs)
            e = hipMemcpyAsync(b->dgraphs, hg.data(), sizeof(DevGraph) * hg.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = upload_lists(ll, b->dmem + gbytes, st, &b->vl, &b->fl);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipFree(b->dmem);
            delete b;
            return hip_error(e, "batch upload");
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
    hipError_t e = run_loop(b->ctx, b->loops, b->dgraphs, b->use_fused ? b->fviews : nullptr, b->vl, b->fl, iters,
                            damping, temperature, (int32_t)b->graphs.size());
    if (e != hipSuccess) return hip_error(e, "batch iteration launch");
    for (lbp_graph *g : b->graphs) {
        g->last_T = temperature;
        ++g->version;
    }
    return LBP_OK;
}

// ---------------------------------------------------------------- samplers
int lbp_sampler_create(lbp_graph *g, int32_t num_samples, lbp_sampler **out) {
    if (!g || !out) return fail(LBP_E_INVALID, "graph or out is NULL");
    if (num_samples < 1 || num_samples > 65535) return fail(LBP_E_INVALID, "num_samples must be in [1, 65535]");
    lbp_sampler *sp = nullptr;
    try {
        HIP_TRY(hipSetDevice(g->ctx->device));
        const int32_t S = num_samples;
        LaunchLists ll;
        std::vector<WorkItem> mids, highs, cols;
        for (int32_t s = 0; s < S; ++s) add_to_lists(ll, s, g->shape, &mids, &highs, &cols);
        finish_lists(ll, mids, highs, cols);
        const size_t vbytes = align256(sizeof(DevGraph) * S), lbytes = lists_bytes(ll);
        const size_t mb = align256(sizeof(float) * g->M), bb = align256(sizeof(float) * g->VB),
                     fb = align256(sizeof(int32_t) * 4);
        const size_t per = mb + 2 * bb + fb;
        const size_t total = vbytes + lbytes + per * (size_t)S;
        sp = new lbp_sampler;
        sp->g = g;
        sp->S = S;
        hipError_t e = hipMalloc((void **)&sp->dmem, total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete sp;
            return fail(LBP_E_OOM, "sampler allocation of " + std::to_string(total) + " bytes failed");
        }
        hipStream_t st = g->ctx->stream;
        std::vector<DevGraph> hv(S, g->host);
        char *p = sp->dmem + vbytes + lbytes;
        for (int32_t s = 0; s < S; ++s, p += per) {
            DevGraph &h = hv[s];
            h.m = h.mo = (float *)p;
            h.B = (float *)(p + mb);
            h.theta = (float *)(p + mb + bb);
            h.flag = (int32_t *)(p + mb + 2 * bb);
            sp->m.push_back(h.m);
            sp->flag.push_back(h.flag);
            // zero panels and idle lanes as in the graph; real entries are
            // rewritten by every run
            if (e == hipSuccess) e = hipMemsetAsync(h.m, 0, sizeof(float) * g->M, st);
            if (e == hipSuccess) e = hipMemsetAsync(h.B, 0, sizeof(float) * g->VB, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h.theta, g->host.theta, sizeof(float) * g->VB, hipMemcpyDeviceToDevice, st);
        }
        sp->views = (DevGraph *)sp->dmem;
        if (e == hipSuccess) e = hipMemcpyAsync(sp->views, hv.data(), sizeof(DevGraph) * S, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = upload_lists(ll, sp->dmem + vbytes, st, &sp->vl, &sp->fl);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipFree(sp->dmem);
            delete sp;
            return hip_error(e, "sampler upload");
        }
        *out = sp;
        return LBP_OK;
    } catch (const std::bad_alloc &) {
        if (sp) {
            if (sp->dmem) (void)hipFree(sp->dmem);
            delete sp;
        }
        return fail(LBP_E_OOM, "host allocation failed");
    }
}

int lbp_sampler_run(lbp_sampler *sp, int32_t iters, float damping, float temperature, const float *noise,
                    int32_t *map_out, float *q_out) {
    if (!sp) return fail(LBP_E_INVALID, "sampler is NULL");
    if (!noise || !map_out) return fail(LBP_E_INVALID, "noise or map_out is NULL");
    std::string why;
    if (!valid_params(iters, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    lbp_graph *g = sp->g;
    HIP_TRY(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    hipError_t e = launch_evidence_perturb(sp->views, sp->S, (int)g->V, g->host.theta, noise, g->VS, st);
    for (int32_t s = 0; s < sp->S && e == hipSuccess; ++s) {
        e = hipMemsetAsync(sp->m[s], 0, sizeof(float) * g->M, st);
        if (e == hipSuccess) e = hipMemsetAsync(sp->flag[s], 0, sizeof(int32_t) * 4, st);
    }
    if (e == hipSuccess)
        e = run_loop(g->ctx, sp->loops, sp->views, nullptr, sp->vl, sp->fl, iters, damping, temperature);
    const TParams P = make_params(damping, temperature);
    const bool maxp = temperature == 0.0f;
    if (e == hipSuccess) e = launch_iteration(sp->views, sp->vl, sp->fl, P, maxp, st, 1);  // beliefs
    for (int32_t s = 0; s < sp->S && e == hipSuccess; ++s)
        e = launch_readout(sp->views + s, g->nvt, maxp, P, q_out ? q_out + (int64_t)s * g->VS : nullptr, 1,
                           map_out + (int64_t)s * g->V, st);
    if (e != hipSuccess) return hip_error(e, "sampler run");
    return LBP_OK;
}

void lbp_sampler_free(lbp_sampler *sp) {
    if (!sp) return;
    (void)hipSetDevice(sp->g->ctx->device);
    (void)hipStreamSynchronize(sp->g->ctx->stream);
    destroy_loops(sp->loops);
    (void)hipFree(sp->dmem);
    delete sp;
}

int lbp_batch_autotune(lbp_batch *b, float damping, float temperature, int32_t reps, int32_t *fused_out) {
    if (!b) return fail(LBP_E_INVALID, "batch is NULL");
    std::string why;
    if (!valid_params(0, damping, temperature, &why)) return fail(LBP_E_INVALID, why);
    if (reps < 1) return fail(LBP_E_INVALID, "reps must be >= 1");
    HIP_TRY(hipSetDevice(b->ctx->device));
    hipStream_t st = b->ctx->stream;
    // the timed launches update every graph's messages: keep and restore them
    int64_t total = 0;
    for (lbp_graph *g : b->graphs) total += g->M;
    float *save = nullptr;
    hipError_t e = hipMalloc((void **)&save, sizeof(float) * (size_t)std::max<int64_t>(1, total));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBP_E_OOM, "autotune message backup");
    }
    int64_t off = 0;
    for (lbp_graph *g : b->graphs) {
        if (e == hipSuccess && g->M)
            e = hipMemcpyAsync(save + off, g->host.m, sizeof(float) * g->M, hipMemcpyDeviceToDevice, st);
        off += g->M;
    }
    int rc = e == hipSuccess ? tune_launches(b->dgraphs, b->vl, b->fl, damping, temperature, reps, st, nullptr)
                             : hip_error(e, "autotune backup");
    if (rc == LBP_OK && b->fviews)
        rc = tune_fused(b->dgraphs, b->fviews, (int32_t)b->graphs.size(), b->vl, b->fl, damping, temperature, reps,
                        st, &b->use_fused);
    off = 0;
    e = hipSuccess;
    for (lbp_graph *g : b->graphs) {
        if (e == hipSuccess && g->M)
            e = hipMemcpyAsync(g->host.m, save + off, sizeof(float) * g->M, hipMemcpyDeviceToDevice, st);
        off += g->M;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    else (void)hipStreamSynchronize(st);
    (void)hipFree(save);
    destroy_loops(b->loops);
    if (rc != LBP_OK) return rc;
    if (e != hipSuccess) return hip_error(e, "autotune restore");
    if (fused_out) *fused_out = b->use_fused;
    return LBP_OK;
}

int lbp_batch_use_fused(lbp_batch *b, int enable) {
    if (!b) return fail(LBP_E_INVALID, "batch is NULL");
    if (enable && !b->fviews) return fail(LBP_E_INVALID, "not every graph of the batch has a fused iteration");
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    destroy_loops(b->loops);
    b->use_fused = enable != 0;
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
