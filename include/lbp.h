/*
 * lbp.h -- C-ABI of liblbp.so: damped, log-domain loopy belief propagation
 * (max-product and sum-product at a temperature) on discrete factor graphs,
 * run by HIP kernels on an AMD Instinct MI355X (gfx950).
 *
 * Method: PGMax (Zhou et al., arXiv 2202.04110).  Messages of a factor graph
 * live in flat edge-state arrays (Sec. "A fully flat array-based LBP
 * implementation"); every iteration recomputes all factor-to-variable
 * messages in parallel from the previous iterate and damps them (Sec.
 * "Package features", citing Pretti 2005); factors are enumeration factors
 * given by their valid configurations (Sec. "Specifying complex factor
 * graphs") or OR / AND logical factors with updates linear in their arity
 * (Sec. "Package features"); variables may have different numbers of states.
 * The paper prints no update equations; this library implements textbook
 * log-domain BP at temperature T with
 *     LSE_T(x) = max x (T = 0),  M + T log sum exp((x - M)/T) (T > 0):
 *   B[v,s] = theta[v,s] + sum_{e in N(v)} m[e,s]
 *   n[e,s] = B[var(e),s] - m[e,s]
 *   u[e_j,s] = LSE_T{ phi_f(c) + sum_l n[e_l,c_l] : c_j = s } - n[e_j,s]
 *   m[e,s] <- d m[e,s] + (1-d) u[e,s], then minus its max over s
 *   q[v,s] = B[v,s] - LSE_T(B[v,:]),  MAP x_v = lowest argmax_s B[v,s]
 * Messages start at 0.  T = 0 is max-product, T = 1 sum-product.
 *
 * Conventions for every function:
 *  - Return value: LBP_OK (0) or a negative LBP_E_* code; lbp_last_error()
 *    returns a message for the calling thread's last failure.  No C++
 *    exception crosses this interface.  On failure, out-parameters are left
 *    untouched and nothing is leaked.
 *  - "Host" pointers are read or written synchronously; "device" pointers are
 *    used in stream order on the context's stream.  The caller owns every
 *    buffer it passes in.
 *  - Work is asynchronous on the context's stream unless stated otherwise;
 *    asynchronous GPU faults surface at the next synchronising call as
 *    LBP_E_HIP.
 *  - Limits: every graph's internal message, belief and potential arrays
 *    must each hold fewer than 2^31 floats (about 8 GiB).
 */
#ifndef LBP_H
#define LBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBP_OK = 0,
    LBP_E_INVALID = -1,     /* bad argument or malformed graph */
    LBP_E_OOM = -2,         /* device or host allocation failed */
    LBP_E_HIP = -3,         /* a HIP runtime call failed */
    LBP_E_STATE = -4,       /* call not valid in the object's current state */
    LBP_E_BUDGET = -5,      /* request larger than the server's memory budget */
    LBP_E_NONFINITE = -6,   /* beliefs contain NaN or infinity */
    LBP_E_UNSUPPORTED = -7  /* valid graph outside the library's kernel limits */
};

enum { LBP_FACTOR_ENUM = 0, LBP_FACTOR_OR = 1, LBP_FACTOR_AND = 2 };

typedef struct lbp_ctx lbp_ctx;
typedef struct lbp_graph lbp_graph;
typedef struct lbp_batch lbp_batch;
typedef struct lbp_sampler lbp_sampler;
typedef struct lbp_server lbp_server;

/*
 * Factor graph description (all host pointers).  The flat-array form of the
 * paper's Sec. "A fully flat array-based LBP implementation": global indices
 * of variable states and of valid factor configurations.
 *
 *  num_vars            V >= 0
 *  var_num_states[V]   states of each variable, 2 <= n <= 64
 *  evidence[VS]        unary log-potentials theta, variable-major (variable v
 *                      owns entries vs_off[v] .. vs_off[v]+n_v-1, vs_off the
 *                      prefix sum of var_num_states); NULL means all zero
 *  num_factors         F >= 0
 *  factor_kind[F]      LBP_FACTOR_ENUM / _OR / _AND
 *  factor_edge_off[F+1] edges of factor f are factor_edge_off[f] ..
 *                      factor_edge_off[f+1]-1; [0] = 0, non-decreasing
 *  edge_var[E]         variable of each edge, E = factor_edge_off[F].  For
 *                      OR / AND the last edge of the factor is the child and
 *                      the others are its parents (at least one); all of
 *                      their variables must be binary
 *  factor_cfg_table[F] configuration table of an enumeration factor, -1 for
 *                      logical factors
 *  num_cfg_tables      NT >= 0
 *  cfg_table_num_cfgs[NT] number of valid configurations; 0 marks a dense
 *                      table holding every joint state of the factor's
 *                      variables in row-major order (last variable fastest)
 *  cfg_table_arity[NT] must equal the arity of every factor using the table
 *  cfg_table_off[NT+1] offsets into cfg_table_states
 *  cfg_table_states    explicit tables: num_cfgs rows of arity states each;
 *                      every state of every slot must appear in at least one
 *                      row (otherwise a message would be -inf)
 *  logpot_off[F+1]     offsets into log_potentials; an enumeration factor
 *                      holds one log-potential per configuration of its
 *                      table, a logical factor none
 *  log_potentials[Tn]  phi_f(c), Tn = logpot_off[F]; must be finite
 *
 * Messages are exchanged (lbp_get_messages / lbp_set_messages) in the flat
 * edge-state order: edge e owns var_num_states[edge_var[e]] consecutive
 * floats, edges in increasing order; ES is the total.
 */
typedef struct lbp_graph_desc {
    int32_t num_vars;
    const int32_t *var_num_states;
    const float *evidence;
    int32_t num_factors;
    const int32_t *factor_kind;
    const int64_t *factor_edge_off;
    const int32_t *edge_var;
    const int32_t *factor_cfg_table;
    int32_t num_cfg_tables;
    const int32_t *cfg_table_num_cfgs;
    const int32_t *cfg_table_arity;
    const int64_t *cfg_table_off;
    const int32_t *cfg_table_states;
    const int64_t *logpot_off;
    const float *log_potentials;
} lbp_graph_desc;

/* Message of the calling thread's last failure ("" if none).  The pointer
 * stays valid until the thread's next lbp_* call. */
const char *lbp_last_error(void);

/* Host-only check of a description; needs no GPU.  sizes_out (may be NULL)
 * receives {V, VS, F, E, ES, Tn}.  Rejects: out-of-range indices, offsets that
 * are not monotone or do not start at 0, n < 2 or n > 64, logical factors on
 * non-binary variables or without a parent, a table whose arity differs from
 * its factor's, a state outside its variable's range, an (edge, state) that
 * no configuration covers, a log-potential count that does not match the
 * table, non-finite evidence or log-potentials.  LBP_E_UNSUPPORTED: a valid
 * graph beyond the kernels' limits (enumeration factors of arity > 8, more
 * than 4096 configurations or more than 64 summed slot states; logical
 * factors of more than 1024 edges). */
int lbp_validate(const lbp_graph_desc *desc, int64_t sizes_out[6]);

/* Host-only diagnostic: compiles the description into the library's internal
 * layout and replays the address arithmetic of every kernel against the
 * sizes of the arrays it touches (no GPU needed; lbp_graph_upload runs the
 * same check).  info_out (may be NULL) receives the internal array sizes
 * {message floats, belief floats, potential floats, factor tiles}.
 * Returns LBP_E_INVALID with a message naming the access on failure. */
int lbp_check_layout(const lbp_graph_desc *desc, int64_t info_out[4]);

/* Context on HIP device `device`.  hip_stream is a hipStream_t the caller
 * keeps alive (e.g. torch.cuda.current_stream().cuda_stream), or NULL for
 * the null stream.  The context owns nothing on the device but its cached
 * launch graphs. */
int lbp_ctx_create(int device, void *hip_stream, lbp_ctx **out);
/* Changes the stream used by later calls on this context. */
int lbp_ctx_set_stream(lbp_ctx *ctx, void *hip_stream);
/* Whether lbp_run_bp / lbp_batch_run replay fixed-iteration loops as
 * captured HIP graphs (default on; the environment variable LBP_NO_GRAPHS=1
 * turns the default off).  Captured and eager launches run the same kernels
 * with the same arguments, so results are identical. */
int lbp_ctx_use_graphs(lbp_ctx *ctx, int enable);
/* Waits for all work queued on the context's stream. */
int lbp_ctx_synchronize(lbp_ctx *ctx);
/* Frees the context; every graph and batch made with it must be freed first. */
void lbp_ctx_destroy(lbp_ctx *ctx);

/* Validates and uploads a graph (Sec. "A fully flat array-based LBP
 * implementation": index arrays computed once, messages in flat arrays).
 * Host arrays are read before return and may be freed afterwards.  The
 * graph owns its device memory until lbp_graph_free.  Messages start at 0.
 * The upload is complete (stream synchronised) when the call returns.  The
 * library may lay the variables out in an order of its own (it renumbers the
 * low-degree parents of logical factors with more than 8 edges); every array
 * that crosses this interface (evidence, beliefs, MAP, messages, gradients,
 * samples) stays in the description's order. */
int lbp_graph_upload(lbp_ctx *ctx, const lbp_graph_desc *desc, lbp_graph **out);
/* Frees a graph after waiting for its queued work. */
void lbp_graph_free(lbp_graph *g);
/* out[8] = {V, VS, F, E, ES, Tn, device_bytes, padded_edge_states}. */
int lbp_graph_sizes(const lbp_graph *g, int64_t out[8]);

/* Replace evidence (VS floats, variable-major) or log-potentials (Tn floats,
 * in log_potentials order) without re-uploading; on_device selects whether
 * `values` is a device pointer (stream-ordered) or a host pointer (read
 * before return).  Device values are not checked for finiteness; non-finite
 * results are reported by the read-out calls. */
int lbp_set_evidence(lbp_graph *g, const float *values, int on_device);
int lbp_set_log_potentials(lbp_graph *g, const float *values, int on_device);

/* Sets every message to 0. */
int lbp_reset_messages(lbp_graph *g);

/* Runs `iters` >= 0 parallel damped iterations from the current messages
 * (Sec. "Package features": parallel updates with damping; the paper's
 * experiments use 200 iterations and damping 0.5).  0 <= damping <= 1 is the
 * weight of the previous message; temperature T >= 0 (0 = max-product).
 * Messages persist, so a second call continues where the first stopped. */
int lbp_run_bp(lbp_graph *g, int32_t iters, float damping, float temperature);

/* Runs iterations as lbp_run_bp until the messages settle: after every
 * check_every >= 1 iterations it measures the residual of the last one, the
 * largest |change| of any edge-state message (NaN or infinity count as not
 * settled), and stops once it is below tol >= 0, or after max_iters >= 0
 * iterations.  iters_done (may be NULL) receives the iterations run and
 * residual_out (may be NULL) the last residual measured (0 if none).  Each
 * check waits for the device; the messages are those of lbp_run_bp with
 * iters_done iterations.  The first call allocates a message-sized
 * workspace kept with the graph (LBP_E_OOM if it does not fit). */
int lbp_run_bp_until(lbp_graph *g, int32_t max_iters, float damping, float temperature, float tol,
                     int32_t check_every, int32_t *iters_done, float *residual_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as lbp_run_bp_until, with the same arguments, the same
 * iterations run and bitwise the same messages and residual, but its
 * workspace (the previous-message copy and the residual partials) lives in a
 * fixed device array of LBP_NOALLOC_SCRATCH_BYTES compiled into the library
 * (each GPU the library runs on holds one until the process ends; its
 * address is looked up once per device by lbp_ctx_create).  The call makes
 * no hipMalloc, hipFree or other allocating call and launches its kernels
 * one by one (no captured loop).  A graph whose workspace exceeds the array
 * (message panel floats rounded up to 256 bytes, plus one float per 256
 * edges, plus one) is refused with LBP_E_UNSUPPORTED before anything runs.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other threads, other contexts, other streams) race and must be
 * serialised by the caller.  Nothing in the array needs to start at zero:
 * each call writes what it reads. */
#define LBP_NOALLOC_SCRATCH_BYTES (64ll << 20)
int lbp_run_bp_until_noalloc(lbp_graph *g, int32_t max_iters, float damping, float temperature, float tol,
                             int32_t check_every, int32_t *iters_done, float *residual_out);

/* Beliefs from the current messages at the temperature of the last run (0
 * before any run), VS floats variable-major: normalised q = B - LSE_T(B) when
 * `normalized`, else B.  MAP: lowest-index argmax of B per variable (V int32;
 * the paper scores MAP inference by the potential of the returned
 * configuration, Sec. "Comparison with existing alternatives").  Outputs on
 * the host synchronise the stream; LBP_E_NONFINITE reports NaN/inf beliefs
 * (the output is still written).  Device outputs are stream-ordered and the
 * non-finite check is then reported by lbp_graph_status. */
int lbp_get_beliefs(lbp_graph *g, float *out, int normalized, int out_on_device);
int lbp_decode_map(lbp_graph *g, int32_t *out, int out_on_device);
/* Synchronises and reports LBP_E_NONFINITE if any read-out since the last
 * call saw a non-finite belief (and clears the flag). */
int lbp_graph_status(lbp_graph *g);

/* Message state in the flat edge-state order (ES floats), for checkpoints and
 * for starting several runs from one state.  The library keeps every message
 * row normalised (its largest state at 0; a row of two states is stored as
 * the one number m1 - m0), so lbp_set_messages normalises the rows of
 * two-state edges it is given: lbp_get_messages then returns them shifted to
 * a largest state of 0.  A shift of a whole row changes no belief or later
 * message (the update is invariant under it), only the rounding. */
int lbp_get_messages(lbp_graph *g, float *out, int on_device);
int lbp_set_messages(lbp_graph *g, const float *values, int on_device);

/*
 * Differentiation through the solver (the paper's Sec. "Exciting new
 * possibilities": LBP as part of an end-to-end differentiable system).
 *
 * lbp_run_bp_record runs like lbp_run_bp (from the current messages) and
 * keeps a checkpoint of the messages every ckpt_every iterations.  It needs
 * temperature > 0 (max-product is not differentiable) and a graph of
 * enumeration factors only (LBP_E_UNSUPPORTED otherwise).  Device memory:
 * about (iters/ckpt_every + ckpt_every + 2) message arrays, owned by the
 * graph until it is freed.
 *
 * lbp_run_bp_backward computes, for the loss L = sum_{v,s} grad_q[v,s] q[v,s]
 * with q the normalised beliefs after the recorded run, dL/dphi into
 * grad_logpot (Tn floats, log_potentials order) and dL/dtheta into
 * grad_evidence (VS floats, or NULL to skip).  All three are device pointers,
 * used in stream order.  The derivative is that of the recorded unrolled
 * iterations (reverse mode: each segment's iterates are recomputed from its
 * checkpoint).  LBP_E_STATE if the graph's messages or inputs changed since
 * the record.  The record stays valid, so backward may be called again.
 */
int lbp_run_bp_record(lbp_graph *g, int32_t iters, float damping, float temperature, int32_t ckpt_every);
int lbp_run_bp_backward(lbp_graph *g, const float *grad_q, float *grad_logpot, float *grad_evidence);

/*
 * Batches (the paper's Sec. "Exciting new possibilities": processing batches
 * of models in parallel).  A batch references graphs uploaded to the same
 * context and advances all of them in shared kernel launches; each graph's
 * arithmetic is the same as when it runs alone, so results are bitwise
 * identical.  The batch does not own its graphs, which must outlive it.
 * Square pairwise factors of 2..8 states share one launch whatever their
 * state count, and so do the variables of up to 8 states, so graphs of
 * different state counts still advance in two launches per iteration.
 */
int lbp_batch_create(lbp_ctx *ctx, lbp_graph *const *graphs, int32_t num_graphs,
                     lbp_batch **out);
int lbp_batch_run(lbp_batch *b, int32_t iters, float damping, float temperature);
/* Fused iterations for a batch whose graphs all have them (see
 * lbp_graph_use_fused): pairs of iterations run as single launches over
 * every graph, with bitwise the same results.  LBP_E_INVALID if a graph has
 * none.  Off by default. */
int lbp_batch_use_fused(lbp_batch *b, int enable);
/* Times the batch's launch shapes as lbp_autotune does for a graph (reps
 * timed launches per candidate) and keeps the fastest; when every graph has
 * fused iterations, also tunes their shapes and switches the batch to fused
 * or two-phase iterations, whichever is faster (*fused_out, if not NULL: 1 if
 * fused).  Every graph's messages are restored before return.  Shapes never
 * change results.  Synchronises the context's stream. */
int lbp_batch_autotune(lbp_batch *b, float damping, float temperature, int32_t reps, int32_t *fused_out);
void lbp_batch_free(lbp_batch *b);

/*
 * Sample batches: many solves of one graph under perturbed evidence in
 * shared launches, for perturb-and-MAP sampling (the method of the blind
 * deconvolution example the paper cites, Sec. "Specifying complex factor
 * graphs"; batches of samples in parallel, Sec. "Exciting new
 * possibilities").  A sampler owns num_samples (1 .. 65535) private sets of
 * messages, beliefs and evidence panels; it shares the graph's structure,
 * potentials and evidence, and the graph must outlive it.
 * lbp_sampler_run: for every sample s, evidence_s = the graph's current
 * evidence + noise[s] (noise: device, num_samples x VS floats, flat
 * variable-state order, summed in FP32), messages from zero, then `iters`
 * iterations at (damping, temperature) and the read-out of sample s:
 * MAP states (map_out: device, num_samples x V int32) and, if q_out is not
 * NULL, normalised beliefs (device, num_samples x VS floats).  Each sample's
 * outputs are bitwise those of the graph run alone with evidence_s set.
 * Perturb-and-MAP: noise drawn i.i.d. from Gumbel(0, 1), scaled, and
 * temperature 0.  The caller draws the noise; asynchronous on the context's
 * stream; the graph's own messages are untouched.  LBP_E_OOM when the
 * sample panels do not fit; LBP_E_INVALID on bad arguments.
 */
int lbp_sampler_create(lbp_graph *g, int32_t num_samples, lbp_sampler **out);
int lbp_sampler_run(lbp_sampler *s, int32_t iters, float damping, float temperature, const float *noise,
                    int32_t *map_out, float *q_out);
void lbp_sampler_free(lbp_sampler *s);

/*
 * Serving with continuous batching.  Requests arrive while others run: a
 * worker thread admits queued requests first-in first-out whenever a slot
 * is free and the server's memory arena (one device allocation of
 * hbm_budget_bytes) has room for the graph, its messages and, for backward
 * requests, the checkpoint workspace.  An uploader thread queues each
 * admitted graph's copies on a copy stream while the compute stream advances
 * every resident graph whose upload is queued by up to steps_per_round
 * iterations per round in shared multi-graph launches (the batch form
 * above); graphs join and leave at round boundaries, and their messages stay
 * resident in between.  Finished graphs are read out on a stream of their
 * own beside the next round.  Results are bitwise equal to lone runs.
 */
typedef struct lbp_completion {
    uint64_t req_id;
    int32_t status;            /* LBP_OK, LBP_E_NONFINITE, LBP_E_STATE (cancelled), other errors */
    int32_t iters_done;        /* iterations run (fewer than asked when a request submitted with
                                * lbp_server_submit_until settled early) */
    int64_t num_vars, num_var_states, num_logpots;
    const float *beliefs;      /* VS normalised beliefs (host), NULL on failure */
    const int32_t *map;        /* V MAP states (host), NULL on failure */
    const float *grad_logpot;  /* Tn gradient (host) for backward requests, else NULL */
    double t_arrival, t_ready, t_admit, t_done;  /* seconds on the server clock: arrival,
                                                  * compiled and checked, admitted, completed */
    float residual;            /* lbp_server_submit_until requests: the last residual measured
                                * (0 if none); other requests: -1 */
    int32_t reserved;
} lbp_completion;

/* Server on ctx's device with an arena of hbm_budget_bytes, at most max_slots
 * resident requests and at most steps_per_round iterations per round.  The
 * server owns its streams and arena; ctx is only read for its device. */
int lbp_server_create(lbp_ctx *ctx, int64_t hbm_budget_bytes, int32_t max_slots, int32_t steps_per_round,
                      lbp_server **out);
/* The same scheduler with a bookkeeping-only executor: no GPU is touched,
 * completions carry zero-filled outputs.  For tests of admission and
 * queueing on hosts without a GPU. */
int lbp_server_create_host_only(int64_t budget_bytes, int32_t max_slots, int32_t steps_per_round, lbp_server **out);
/* Seconds since the server was created (the clock of every timestamp). */
double lbp_server_clock(const lbp_server *s);
/* Queues a request.  Its host arrays are copied before return (their
 * lengths are read from the offsets, so they must be as long as the
 * description says); validation (lbp_validate's checks) and compilation run
 * on the server's prep threads, a failing request completes with status
 * LBP_E_INVALID or LBP_E_UNSUPPORTED, and admission stays first-in
 * first-out.  Null arrays, negative counts and bad parameters are rejected
 * at once with LBP_E_INVALID.  grad_q
 * (host, VS floats) != NULL asks for the gradient of sum(grad_q * q) w.r.t.
 * the log-potentials (T > 0, enumeration factors only), with checkpoints
 * every ckpt_every iterations.  t_arrival: the request's arrival time on the
 * server clock (its latency is measured from it), or < 0 for "now".  A
 * request that alone needs more than the budget completes with status
 * LBP_E_BUDGET. */
int lbp_server_submit(lbp_server *s, const lbp_graph_desc *desc, int32_t iters, float damping, float temperature,
                      const float *grad_q, int32_t ckpt_every, double t_arrival, uint64_t req_id);
/* Queues a forward request that stops once its messages settle, as
 * lbp_run_bp_until(max_iters, damping, temperature, tol, check_every) on the
 * graph alone: the residual of the last iteration is measured whenever the
 * request's own iteration count reaches a multiple of check_every (or
 * max_iters), and the request leaves at that round boundary once it is below
 * tol, freeing its slot and memory for queued requests.  Rounds never step
 * over a request's check points, so the iterations run, the messages, the
 * beliefs and the residual are bitwise those of the lone lbp_run_bp_until
 * call whatever else is resident.  The completion reports iters_done and the
 * residual.  The previous-message workspace (a message-sized buffer) counts
 * against the budget.  tol must be finite and >= 0, check_every >= 1; other
 * arguments as for lbp_server_submit (no gradient). */
int lbp_server_submit_until(lbp_server *s, const lbp_graph_desc *desc, int32_t max_iters, float damping,
                            float temperature, float tol, int32_t check_every, double t_arrival, uint64_t req_id);
/* Marks a queued or resident request cancelled; it completes with
 * LBP_E_STATE at the next round boundary. */
int lbp_server_cancel(lbp_server *s, uint64_t req_id);
/* Moves up to max finished requests into out[0 .. *n_out-1].  Their output
 * pointers stay valid until the next poll or lbp_server_destroy. */
int lbp_server_poll(lbp_server *s, lbp_completion *out, int32_t max, int32_t *n_out);
/* Waits until every accepted request has finished (LBP_E_STATE on timeout). */
int lbp_server_drain(lbp_server *s, double timeout_s);
/* out[18] = {accepted, finished, completed, rejected for the budget, failed,
 * cancelled, rounds, resident now, queued now, max resident, arena peak bytes,
 * worker busy microseconds, of which in rounds (launch + wait), preparation
 * microseconds summed over the preparation threads, preparation threads,
 * worker microseconds in admissions (handing requests to the uploader), in
 * enqueueing rounds (launch lists and kernels), in read-outs of finished
 * requests}. */
int lbp_server_stats(lbp_server *s, int64_t out[18]);
/* Stops the worker (queued and resident requests are dropped) and frees
 * everything. */
void lbp_server_destroy(lbp_server *s);

/*
 * Launch shapes and the autotuner.  A graph's work runs as a few launch
 * groups (the variable phase, then one group per factor shape class).  Each
 * group has a shape: wavefronts per block (1, 2 or 4; the variable phase and
 * generic enumeration groups are fixed at 4) and whether blocks are remapped
 * so that each of the 8 XCDs takes a contiguous range of tiles.  Shapes never
 * change any element's arithmetic, so results are identical whatever the
 * shape.  lbp_autotune times every candidate shape of every group with HIP
 * events inside whole two-phase iterations (reps iterations each, the other
 * groups at their current shapes, two passes over the groups; messages saved
 * and restored), so what one phase leaves in the caches for the next counts,
 * and keeps the fastest; best_ms_out (may be NULL) receives, per group, the
 * iteration time with its chosen shape.  lbp_graph_get_launch returns
 * {phase (0 variable, 1 factor), kind, a, b, waves per block, swizzle, work
 * items, fused waves per block, fused variant} for group i.
 */
int lbp_graph_num_launches(const lbp_graph *g, int32_t *n_out);
int lbp_graph_get_launch(const lbp_graph *g, int32_t i, int32_t out[9]);
int lbp_graph_set_launch(lbp_graph *g, int32_t i, int32_t waves_per_block, int32_t swizzle);
/* Shape of the fused variant of factor launch i (see lbp_graph_use_fused);
 * lbp_graph_get_launch returns it in out[7], out[8].  variant: bit 0 = the
 * XCD swizzle; bit 1 = each wavefront loads its factors' tables before
 * gathering their variables' beliefs instead of after (more loads in flight,
 * more registers, fewer wavefronts resident: it pays when the graph streams
 * from HBM rather than sitting in the last-level cache).  Bitwise the same
 * results for every variant. */
int lbp_graph_set_fused_launch(lbp_graph *g, int32_t i, int32_t waves_per_block, int32_t variant);
int lbp_autotune(lbp_graph *g, float damping, float temperature, int32_t reps, float *best_ms_out);
/* Fused iterations: for a graph whose variables all have at most 16 edges and
 * 16 states and whose factors are all dense pairwise with equal slot sizes,
 * a whole iteration can run in the factor launch (each factor recomputes its
 * variables' beliefs from the previous messages, with the variable phase's
 * exact arithmetic; messages alternate between two buffers and always end in
 * the graph's own).  Results are bitwise identical either way; speed depends
 * on the graph and cache sizes, so lbp_autotune switches it on only when it
 * measures faster.  Off by default.  out = {available, in use}. */
int lbp_graph_use_fused(lbp_graph *g, int enable);
int lbp_graph_fused_state(const lbp_graph *g, int32_t out[2]);
/* Resident solver (Sec. "Package features": the same parallel damped
 * updates): a graph whose messages and beliefs fit in one workgroup's LDS
 * (the device's limit; index arrays, evidence and tables join them while
 * they fit), whose
 * variables have at most 64 edges and whose factors are all pairwise or
 * OR/AND of at most 256 edges is solved by lbp_run_bp in one workgroup that
 * keeps messages and beliefs in on-chip memory for all iterations, with the
 * same per-element arithmetic as launched iterations (bitwise identical
 * results).  One workgroup works through the tiles that launched iterations
 * spread over the whole device, so it pays only for the smallest graphs:
 * off by default, lbp_autotune switches it on when it measures faster.
 * Enabling it where it does not apply is LBP_E_INVALID.  Other entry points
 * (batches, lbp_run_bp_until, records) always launch.  out = {applies, in
 * use}. */
int lbp_graph_use_resident(lbp_graph *g, int enable);
int lbp_graph_resident_state(const lbp_graph *g, int32_t out[2]);

/* Diagnostic timing: runs `reps` launches of one phase of an iteration on the
 * current messages and returns the mean time per launch (per iteration for
 * phases 2 and 3) in milliseconds, measured with HIP events on the context's
 * stream.  phase 0 = variable (belief) kernels, 1 = factor kernels (in
 * place), 2 = two-phase iterations, 3 = fused iterations (graphs whose
 * variables all have at most 16 edges and 16 states and whose factors are
 * all dense pairwise with equal slot sizes; lbp_run_bp uses them for such
 * graphs, with bitwise the same results).  Phases 1-3 update the messages. */
int lbp_time_phase(lbp_graph *g, int32_t phase, int32_t reps, float damping, float temperature,
                   float *ms_out);

/* Diagnostic: average time in milliseconds of one launch of a plain
 * streaming kernel (float4 accesses, grid-stride, `blocks` workgroups of 256
 * threads) over `reps` launches after one warm-up, HIP events on the
 * context's stream.  It sets the bandwidth an ordinary kernel reaches on the
 * device, beside the nominal peak.  kind 0: read `bytes` of src (device,
 * contents should be zeros; dst, device, receives at most one float);
 * 1: copy `bytes` from src to dst; 2: write `bytes` of dst (src unused, may
 * be NULL); 3: read `bytes` of src and write bytes / 5 of dst (five reads per
 * write, about the mix of an iteration's factor launches).  bytes > 0 must be
 * a multiple of 16 (of 80 for kind 3); pointers 16-byte aligned.  The call
 * synchronises on its end event. */
int lbp_bandwidth_probe(lbp_ctx *ctx, int32_t kind, const void *src, void *dst, int64_t bytes, int32_t blocks,
                        int32_t reps, float *ms_out);

#ifdef __cplusplus
}
#endif

#endif /* LBP_H */
