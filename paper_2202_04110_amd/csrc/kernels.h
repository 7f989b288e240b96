// Launchers of the HIP kernels (kernels.hip).  Each returns the HIP error of
// the launch; item arrays and graph arrays are device pointers.
#pragma once

#include <hip/hip_runtime.h>

#include "lbp_internal.h"

namespace lbp {

// Per-launch constants of an iteration at damping d and temperature T.
struct TParams {
    float d, omd;  // weight of the previous message and 1 - d
    float T, invT;
    float c, r;    // log2(e) / T and T ln 2 (LSE_T in base 2)
};

TParams make_params(float damping, float temperature);

// A graph's launch list for the resident solver (passed by value): variable
// launches first (a: state bucket; n low tiles then n_mid wavefront items),
// then factor launches (kind, a, b as launched; n items).
struct SolveLaunch {
    int32_t kind, a, b, n, n_mid, pad;
    const WorkItem *items;
};
constexpr int kSolveLaunchesMax = 12;
// Graph arrays the resident solver may hold in LDS, in placement order:
// messages and beliefs always, then (each while it fits) the index arrays
// and tile descriptors that start every tile's load chain, the evidence, the
// potential tables.
enum SolveArray : int32_t {
    SA_M, SA_B, SA_VEDGE, SA_FVB, SA_HEDGE, SA_VNS, SA_VTILE, SA_FTILE, SA_HVAR, SA_THETA, SA_PHI, SA_COUNT
};
struct SolvePlan {
    int32_t nv = 0, nf = 0;
    int32_t words[SA_COUNT] = {};  // size of each array in 4-byte words
    uint32_t lds_mask = 0;         // arrays copied into LDS
    int32_t lds_words = 0;         // their total, each rounded up to 4 words (16-byte aligned placements)
    SolveLaunch l[kSolveLaunchesMax];
};
__host__ __device__ constexpr int64_t solve_words_aligned(int64_t w) { return (w + 3) & ~int64_t(3); }

// Launch shape of a wavefront-per-item kernel: wavefronts per block (1, 2 or
// 4), whether blocks are remapped so each XCD takes a contiguous range, and
// (fused pairwise launches only) whether tables are loaded before the belief
// gathers.  None changes any element's arithmetic.
struct LaunchShape {
    int wpb = 4;
    int swizzle = 0;
    int early = 0;
};

// Buffers of the reverse sweep (message panels A, nbar; belief panel Bbar;
// potential panel phibar).
struct AdjBufs {
    float *A;
    float *nbar;
    const float *Bbar;
    float *phibar;
};

// Variable phase: items = n_low low tiles, then n_mid and n_high variables
// (indices into the graph's hvar list); bucket >= states of every low lane.
hipError_t launch_belief(const DevGraph *gs, const WorkItem *items, int n_low, int n_mid, int n_high, int bucket,
                         const LaunchShape &S, hipStream_t st);
// fused: one whole iteration in the factor launch (square classes only; see
// pair_tile), reading G.m and writing G.mo.
hipError_t launch_pair(const DevGraph *gs, const WorkItem *items, int n, int na, int nb, bool maxp,
                       const TParams &P, const LaunchShape &S, hipStream_t st, bool fused = false);
// Logical tiles: wide = false for lane tiles and factors of <= 256 edges,
// true for factors of 257..1024 edges.
hipError_t launch_logical(const DevGraph *gs, const WorkItem *items, int n, bool wide, bool maxp, const TParams &P,
                          const LaunchShape &S, hipStream_t st);
// Generic classes.  lds_code -N: dense three-way classes with N (2..4)
// states per slot, in registers; 0: the kernel with LDS for the largest
// class; otherwise gen_lds_code(rows bytes, summed slot states) of the
// classes in the launch, which sizes its dynamic LDS.
hipError_t launch_gen(const DevGraph *gs, const WorkItem *items, int n, bool maxp, const TParams &P, int lds_code,
                      hipStream_t st);
// Read-out of a single graph (gs[0]).
// `iters` iterations of one small graph in a single workgroup holding the
// arrays of plan.lds_mask in LDS (plan.lds_words words, which must include
// the messages and beliefs); no block-per-variable items, pairwise and lane
// logical factor launches only (hipErrorInvalidValue otherwise).  Bitwise the
// same as launched two-phase iterations.
hipError_t launch_solve_resident(const DevGraph *g, const SolvePlan &plan, int32_t iters, bool maxp, const TParams &P,
                                 hipStream_t st);
// Largest LDS allocation of one workgroup on `device`, in bytes (0 if unknown).
int32_t solve_lds_limit(int device);
hipError_t launch_readout(const DevGraph *gs, int nvtiles, bool maxp, const TParams &P, float *q, int normalized,
                          int32_t *map, hipStream_t st);
// Read-out of one graph inside a multi-graph launch: its normalised beliefs
// (VS floats, flat order) and MAP (V ints) go to q and map, which may be
// page-locked host memory; *flag is set to 1 on a non-finite belief (the
// caller clears it first).  The beliefs B must be current.
struct ReadJob {
    const DevGraph *g;
    float *q;
    int32_t *map;
    int32_t *flag;
    TParams P;
    int32_t ntiles, maxp;
};
hipError_t launch_readout_multi(const ReadJob *jobs, int n, int max_tiles, hipStream_t st);
hipError_t launch_msgs_out(const DevGraph *gs, int E, float *out, hipStream_t st);
hipError_t launch_msgs_in(const DevGraph *gs, int E, const float *in, hipStream_t st);
hipError_t launch_evidence_in(const DevGraph *gs, int V, const float *in, hipStream_t st);
// Residual of the last iteration of a single graph (gs[0]): out[0] = max over
// edge-state entries of |m - mprev| (non-finite as infinity); partial holds
// residual_blocks(E) floats.
int residual_blocks(int E);
hipError_t launch_residual(const DevGraph *gs, int E, const float *mprev, float *partial, float *out, hipStream_t st);
// Fixed scratch of the entry point that allocates nothing: a file-scope
// device array in kernels.hip (every GPU the library runs on holds its own
// copy until the process ends).  noalloc_scratch_address returns its device
// address on `device`, which must be the current device; the first call per
// device looks it up (hipGetSymbolAddress), later calls return the kept value.
// Bandwidth probes (plain streaming kernels): kind 0 reads `bytes` of src
// (dst receives at most one float), 1 copies `bytes` from src to dst, 2
// writes `bytes` of dst, 3 reads `bytes` of src and writes bytes / 5 of dst.
// bytes is a multiple of 16 (of 80 for kind 3); pointers 16-byte aligned.
hipError_t launch_stream_probe(int kind, const void *src, void *dst, int64_t bytes, int blocks, hipStream_t st);
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch_address(int device, float **out);
// One graph's convergence check inside a multi-graph launch: g is the
// device copy of its descriptor, mprev (M floats, M a multiple of 4, 16-byte
// aligned) receives its messages before the checked iteration, partial holds
// residual_blocks(E) floats, and the residual goes to out[slot].
struct ConvJob {
    const DevGraph *g;
    float *mprev;
    float *partial;
    int32_t E, M, slot, pad;
};
// mprev = messages for every job (max_M: the largest M); then, after the
// iteration, out[slot] = residual for every job (max_E: the largest E).
hipError_t launch_save_multi(const ConvJob *jobs, int n, int max_M, hipStream_t st);
hipError_t launch_residual_multi(const ConvJob *jobs, int n, int max_E, float *out, hipStream_t st);
// Sample s (0 <= s < S) of views: evidence = base panel + noise[s * VS + ...].
hipError_t launch_evidence_perturb(const DevGraph *views, int S, int V, const float *base, const float *noise,
                                  int64_t VS, hipStream_t st);
hipError_t launch_logpot_in(const DevGraph *gs, int F, const float *in, hipStream_t st);

// adjoint
hipError_t launch_pair_adj(const DevGraph *gs, const WorkItem *items, int n, int na, int nb, const TParams &P,
                           const AdjBufs &J, hipStream_t st);
hipError_t launch_gen_adj(const DevGraph *gs, const WorkItem *items, int n, const TParams &P, const AdjBufs &J,
                          hipStream_t st);
hipError_t launch_readout_adj(const DevGraph *gs, int nvtiles, const TParams &P, const float *gq, float *bbar,
                              float *thetabar, hipStream_t st);
hipError_t launch_accumulate(float *y, const float *x, int64_t n, hipStream_t st);
hipError_t launch_logpot_out(const DevGraph *gs, int F, const float *panel, float *out, hipStream_t st);
hipError_t launch_evidence_out(const DevGraph *gs, int V, const float *panel, float *out, hipStream_t st);

}  // namespace lbp
