// Internal runtime of liblbp.so shared by the C-ABI (api.cpp) and the serving
// loop (server.cpp): contexts, uploaded graphs, launch lists, the iteration
// driver, read-out and the reverse sweep.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbp.h"
#include "compile.h"
#include "kernels.h"

namespace lbp {

// Thread-local last error: set_error returns `code` so callers can
// `return set_error(...)`.
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);
const char *last_error();

#define HIP_TRY(expr)                                          \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return ::lbp::hip_error(e_, #expr); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
bool valid_params(int32_t iters, float d, float T, std::string *why);

// A set of work items launched by one kernel.
struct Launch {
    int32_t kind;     // -1 variable phase, TK_* factor kernels
    int32_t a, b;     // variable phase: state bucket; PAIR: slot state counts
    int32_t n;        // items (variable phase: low tiles)
    WorkItem *items;  // device
    int32_t n_mid = 0, n_high = 0;  // variable phase: wavefront- and block-per-variable items after the tiles
    LaunchShape shape;              // chosen by lbp_autotune (variable phase: swizzle only)
    LaunchShape fshape;             // shape of the fused variant of a pairwise launch
};

// Host-side launch lists of one graph or of a set of graphs (graph index gi
// in each work item), before upload.
struct LaunchLists {
    std::vector<int32_t> vbucket;                 // variable launches: state bucket
    std::vector<std::vector<WorkItem>> vitems;    // tiles, then (first launch only) mids, column groups, highs
    int32_t n_mid = 0, n_high = 0;                // n_high counts column groups and single block-path variables
    std::vector<FGroup> fshape;                   // factor launches: kind, a, b
    std::vector<std::vector<WorkItem>> fitems;
};

struct GraphShape;  // below
void add_to_lists(LaunchLists &ll, int32_t gi, const GraphShape &s, std::vector<WorkItem> *mids,
                  std::vector<WorkItem> *highs, std::vector<WorkItem> *cols);
// merge (lists of several graphs): square pairwise launches of 2..8 states
// become one mixed launch (a = b = 0; each wavefront takes its tile's own
// state count), and variable launches of buckets up to 8 become one launch
// of the largest bucket, so graphs of different state counts share launches.
// The arithmetic of each element is unchanged.  Block-path items: column
// groups first (the longest), ordered so that consecutive groups of a graph,
// whose edge rows share cache lines, run on one XCD; then single variables.
void finish_lists(LaunchLists &ll, std::vector<WorkItem> &mids, std::vector<WorkItem> &highs,
                  std::vector<WorkItem> &cols, bool merge = false);
// Device bytes of the lists' work items (one 256-aligned piece per launch).
size_t lists_bytes(const LaunchLists &ll);
// Launch descriptors of lists whose items sit at device address `mem`.
void describe_lists(const LaunchLists &ll, char *mem, std::vector<Launch> *vl, std::vector<Launch> *fl);
// Writes the lists' items at host address `host` in the same arrangement.
void pack_lists(const LaunchLists &ll, char *host);
// Copies the lists into `mem` on `st` and fills the launch descriptors.
hipError_t upload_lists(const LaunchLists &ll, char *mem, hipStream_t st, std::vector<Launch> *vl,
                        std::vector<Launch> *fl);

hipError_t launch_iteration(const DevGraph *gs, const std::vector<Launch> &vl, const std::vector<Launch> &fl,
                            const TParams &P, bool maxp, hipStream_t st, int phases = 3);
// `iters` iterations of fusable graphs: pairs of fused iterations through
// the second message buffers (fused[g]: graph g's m -> m2 view,
// fused[stride + g]: its m2 -> m view; stride = the number of graphs), then
// one two-phase in-place iteration on gs if iters is odd, so the messages end
// in each graph's own buffer.  Bitwise the same as two-phase iterations.
hipError_t launch_loop(const DevGraph *gs, const DevGraph *fused, const std::vector<Launch> &vl,
                       const std::vector<Launch> &fl, int32_t iters, const TParams &P, bool maxp, hipStream_t st,
                       int32_t fused_stride = 1);

// A captured fixed-iteration loop, replayed with hipGraphLaunch.
struct CachedLoop {
    int32_t iters;
    float d, T;
    hipGraphExec_t exec;
};
void destroy_loops(std::vector<CachedLoop> &v);

// The groups of a compiled graph needed to build launch lists.
struct GraphShape {
    std::vector<FGroup> fgroups;
    std::vector<VGroup> vgroups;
    std::vector<int32_t> mids, highs, cols;
};

}  // namespace lbp

struct lbp_ctx {
    int device;
    hipStream_t stream;             // the caller's stream (borrowed)
    hipStream_t capture = nullptr;  // private stream used only to record launch graphs
    bool use_graphs = true;
};

struct lbp_graph {
    lbp_ctx *ctx = nullptr;
    int64_t V = 0, VS = 0, F = 0, E = 0, ES = 0, Tn = 0, M = 0, VB = 0, P = 0;
    int32_t nvt = 0;
    char *dmem = nullptr;
    size_t dbytes = 0;
    bool owns_memory = true;
    lbp::DevGraph host{};             // device pointers, host copy
    lbp::DevGraph *dgraph = nullptr;  // device copy
    lbp::DevGraph *fused = nullptr;   // device [2]: fused views over the two message buffers, or null
    float *m2 = nullptr;              // the second message buffer of a fusable graph (device), or null
    bool use_fused = false;           // lbp_run_bp runs fused iterations (chosen by the autotuner)
    bool resident_ok = false;         // small enough for the resident solver (plan below)
    bool use_resident = false;        // lbp_run_bp runs the resident solver (chosen by the autotuner)
    lbp::SolvePlan plan;
    float *q_tmp = nullptr;           // VS
    int32_t *map_tmp = nullptr;       // V
    std::vector<lbp::Launch> vl, fl;  // the graph's own launches
    lbp::GraphShape shape;
    float last_T = 0.0f;
    std::vector<lbp::CachedLoop> loops;
    bool has_logical = false;
    uint64_t version = 0;  // bumped by every call that changes messages or inputs
    char *conv = nullptr;  // lbp_run_bp_until workspace: previous messages, partial and final residuals
    // reverse-sweep workspace and the record it belongs to
    struct Adjoint {
        bool valid = false;
        uint64_t version = 0;
        int32_t iters = 0, k = 0, nseg = 0;
        float d = 0.0f, T = 0.0f;
        char *dmem = nullptr;
        size_t bytes = 0;
        bool owns_memory = true;
        float *ckpt = nullptr, *seg = nullptr, *A = nullptr, *nbar = nullptr, *Bbar = nullptr, *Bt = nullptr,
              *zeros = nullptr, *thetabar = nullptr, *phibar = nullptr;
        lbp::DevGraph *views = nullptr;  // [0, k): iterates in seg; [k]: current messages; [k+1]: adjoint view
    } adj;
};

struct lbp_batch {
    lbp_ctx *ctx = nullptr;
    std::vector<lbp_graph *> graphs;
    char *dmem = nullptr;
    lbp::DevGraph *dgraphs = nullptr;
    lbp::DevGraph *fviews = nullptr;  // device [2 * graphs]: every graph's fused views, when all are fusable
    bool use_fused = false;
    std::vector<lbp::Launch> vl, fl;
    std::vector<lbp::CachedLoop> loops;
};

struct lbp_sampler {
    lbp_graph *g = nullptr;
    int32_t S = 0;
    char *dmem = nullptr;
    lbp::DevGraph *views = nullptr;  // device [S]: the graph with sample s's messages, beliefs, evidence
    std::vector<float *> m;          // sample s's message panels (device)
    std::vector<int32_t *> flag;     // sample s's read-out flags (device)
    std::vector<lbp::Launch> vl, fl;
    std::vector<lbp::CachedLoop> loops;
};

namespace lbp {

// Runs `iters` iterations on the context's stream: through a cached captured
// graph when enabled (same kernels and arguments as eager launches), else by
// launching each kernel.
// fused: the graph's fused views (nullptr for two-phase iterations).
hipError_t run_loop(lbp_ctx *ctx, std::vector<CachedLoop> &cache, const DevGraph *gs, const DevGraph *fused,
                    const std::vector<Launch> &vl, const std::vector<Launch> &fl, int32_t iters, float d, float T,
                    int32_t fused_stride = 1);

// Device bytes an uploaded layout occupies (with_fused: plus the second
// message buffer and views of the fused iteration, if the layout allows it).
size_t graph_device_bytes(const HostLayout &L, bool with_fused);
// Host image of a graph's device data: the layout's arrays and launch lists
// packed in device order (graph_image_bytes(L) bytes, written by
// graph_fill_image), uploaded with one copy.
size_t graph_image_bytes(const HostLayout &L);
// Writes the image.  A layout compiled without its panels (compile_desc with
// fill = false) gets the evidence of `d` as given (checked by compile_desc);
// its log-potentials as given travel in a buffer of the caller's, checked by
// the caller, and are not part of the image.
int graph_fill_image(const HostLayout &L, char *image, const lbp_graph_desc *d = nullptr);
// Creates a graph from a compiled (and checked) layout.  mem: a 256-aligned
// region of graph_device_bytes(L, with_fused) bytes the caller owns, or
// nullptr to allocate.  image: the layout's host image, or nullptr to build
// one here (the graph's device descriptor is written into it); a layout
// compiled without its panels needs its image and, when it has any, its
// L.Tn log-potentials as given in raw_lp (NaN and infinity already refused).
// Copies run on `st`, and the call waits for them unless wait is false and
// the caller brings the image: then the image and raw_lp must outlive the
// copies and work on other streams must wait for `st` before using the graph.
int graph_create(lbp_ctx *ctx, const HostLayout &L, bool with_fused, char *mem, hipStream_t st, lbp_graph **out,
                 char *image = nullptr, bool wait = true, const float *raw_lp = nullptr);
void graph_destroy(lbp_graph *g);
// The resident solver's plan of a graph's launch lists, if the graph fits it
// (messages and beliefs within limit_words 4-byte words of LDS, no
// block-per-variable items, pairwise and lane logical factor launches only);
// the other arrays are placed in LDS in SolveArray order while they fit.
bool make_solve_plan(const std::vector<Launch> &vl, const std::vector<Launch> &fl, const HostLayout &L,
                     int64_t limit_words, SolvePlan *plan);

// Read-out (beliefs and/or MAP) on `st`; host outputs are copied with
// hipMemcpyAsync and are complete once `st` is synchronised.
int graph_readout(lbp_graph *g, float *q, int normalized, int32_t *map, bool out_on_device, hipStream_t st);

// Reverse sweep.
size_t adjoint_bytes(int64_t M, int64_t VB, int64_t P, int32_t iters, int32_t ckpt_every);
// Sets up the workspace (mem: adjoint_bytes(...) bytes owned by the caller,
// or nullptr to allocate) and the views for a record of (iters, d, T, k);
// marks the record invalid until adjoint_finish_record.  The views are
// staged in `staging` when given (host memory the caller keeps until the
// copies queued on st have completed; nothing waits here), else in a local
// buffer and st is synchronised.
int adjoint_prepare(lbp_graph *g, int32_t iters, float d, float T, int32_t ckpt_every, char *mem, hipStream_t st,
                    std::vector<DevGraph> *staging = nullptr);
// Copies the current messages into checkpoint `seg` on `st`.
int adjoint_checkpoint(lbp_graph *g, int32_t seg, hipStream_t st);
void adjoint_finish_record(lbp_graph *g);
int adjoint_backward(lbp_graph *g, const float *grad_q, float *grad_logpot, float *grad_evidence, hipStream_t st);

}  // namespace lbp
