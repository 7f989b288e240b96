// HIP kernels of one damped log-domain LBP iteration on gfx950 (CDNA4).
//
// An iteration (parallel updates with damping, PGMax Sec. "Package
// features") runs in two phases:
//   variable phase  B[v,s] = theta[v,s] + sum_{e in N(v)} m[e,s]
//                   (segmented sum over the variable's edge rows, edges in
//                   increasing order, no atomics)
//   factor phase    n = B[var(e)] - m[e]  (formed on the fly, never stored),
//                   factor-to-variable update u (max / LSE_T over the
//                   factor's configurations, or the OR/AND closed forms),
//                   then m <- d m + (1-d) u and m -= max_s m, written in
//                   place.  Each message row is read and written by the one
//                   lane that owns its factor, after the variable phase has
//                   consumed the old values, so no barrier is needed inside
//                   the phase.
// The work is memory-bound: there is no dense contraction, hence no MFMA.
// Data sit in 64-lane panels (lbp_internal.h) so that a wavefront's loads
// and stores are unit-stride 256-byte accesses.
//
// Every per-element result is computed by one device function in a fixed
// order whichever kernel, batch or launch shape runs it, and the library is
// built with -ffp-contract=off, so a graph gives the same bits alone and in a
// batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "kernels.h"

// Scratch of lbp_run_bp_until_noalloc: the previous-message copy and the
// residual partials live here instead of in memory the library allocates.
// In host code this name is a host-side stand-in, not a device address: the
// address is looked up per device (noalloc_scratch_address) and only that
// value is handed to kernels and copies.
static __device__ __align__(256) float scratch[lbp::kNoAllocScratchBytes / sizeof(float)];

namespace lbp {

namespace {

__device__ __forceinline__ int wave_index(int waves_per_block) {
    return __builtin_amdgcn_readfirstlane((int)(blockIdx.x * waves_per_block + (threadIdx.x >> 6)));
}

// The graph's arrays as global-address-space pointers.  Kernels take the
// descriptor by pointer, so its pointer fields reach device code as generic
// pointers, and every access through them would be a flat access (64-bit
// VGPR addresses, waits shared with scalar loads).  Launched kernels read
// the descriptor into this view once and pass it to the tile functions
// (templates on the view type), whose loads and stores then use global
// instructions with a scalar base; the resident solver, whose descriptor
// points into LDS, passes the generic descriptor itself.
// (The host compilation pass of this file generates no device code and has
// no such address space: there the view holds plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T *;
#else
template <class T>
using gptr = T *;
#endif
struct GGraph {
    gptr<float> m, mo, B, theta, phi;
    gptr<const FTile> ftile;
    gptr<const int32_t> fvb, fvar, faff;
    gptr<const VTile> vtile;
    gptr<const int32_t> vedge, vns;
    gptr<const HVar> hvar;
    gptr<const int32_t> hedge;
    gptr<const GenClass> gcls;
    gptr<const uint8_t> grows;
    gptr<const int32_t> edge_maddr;
    gptr<const int64_t> es_off, vs_off;
    gptr<const int32_t> vn, fac_phi, vext;
    gptr<const int64_t> lp_off;
    gptr<int32_t> flag;
    int32_t V, E, F, zero_addr, raw_msgs;
};
template <class T>
__device__ __forceinline__ gptr<T> as_global(T *p) {
    return (gptr<T>)p;
}
__device__ __forceinline__ GGraph glob(const DevGraph &d) {
    GGraph g;
    g.m = as_global(d.m);
    g.mo = as_global(d.mo);
    g.B = as_global(d.B);
    g.theta = as_global(d.theta);
    g.phi = as_global(d.phi);
    g.ftile = as_global(d.ftile);
    g.fvb = as_global(d.fvb);
    g.fvar = as_global(d.fvar);
    g.faff = as_global(d.faff);
    g.vtile = as_global(d.vtile);
    g.vedge = as_global(d.vedge);
    g.vns = as_global(d.vns);
    g.hvar = as_global(d.hvar);
    g.hedge = as_global(d.hedge);
    g.gcls = as_global(d.gcls);
    g.grows = as_global(d.grows);
    g.edge_maddr = as_global(d.edge_maddr);
    g.es_off = as_global(d.es_off);
    g.vs_off = as_global(d.vs_off);
    g.vn = as_global(d.vn);
    g.fac_phi = as_global(d.fac_phi);
    g.vext = as_global(d.vext);
    g.lp_off = as_global(d.lp_off);
    g.flag = as_global(d.flag);
    g.V = d.V;
    g.E = d.E;
    g.F = d.F;
    g.zero_addr = d.zero_addr;
    g.raw_msgs = d.raw_msgs;
    return g;
}

// Workgroups are dealt to the 8 XCDs round-robin.  With swizzling, block b of
// n maps to a logical block such that each XCD runs one contiguous range of
// logical blocks (neighbouring tiles then share that XCD's L2).  A bijection
// on [0, n): the last n mod 8 blocks keep their index.
constexpr int kXcds = 8;
__device__ __forceinline__ int swizzle_block(int b, int n) {
    const int per = n / kXcds;
    if (b >= per * kXcds) return b;
    return (b % kXcds) * per + b / kXcds;
}

// Work item of this wavefront: blockDim.x / 64 wavefronts per block.
__device__ __forceinline__ int wave_item(int swz) {
    const int wpb = blockDim.x >> 6;
    const int b = swz ? swizzle_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    return __builtin_amdgcn_readfirstlane(b * wpb + (int)(threadIdx.x >> 6));
}
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Inclusive prefix sum over the 64 lanes of a wavefront with DPP moves:
// shifts by 1, 2, 4, 8 inside each row of 16 lanes (lanes without a source
// add 0), then row 15's and row 31's values carried into the rows above.
// A fixed sequence of additions, so every wavefront gets the same bits.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_take(float y) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), CTRL, ROW_MASK, 0xf, true));
}
// the same move, lanes without a source (or masked off) reading `fill`
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_take_or(float y, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(y), CTRL, ROW_MASK, 0xf,
                                                      false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_take_or_i(int y, int fill) {
    return __builtin_amdgcn_update_dpp(fill, y, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ float wave_incl_scan(float y) {
    y += dpp_take<0x111, 0xf>(y);  // row_shr:1
    y += dpp_take<0x112, 0xf>(y);  // row_shr:2
    y += dpp_take<0x114, 0xf>(y);  // row_shr:4
    y += dpp_take<0x118, 0xf>(y);  // row_shr:8
    y += dpp_take<0x142, 0xa>(y);  // row_bcast:15 into rows 1 and 3
    y += dpp_take<0x143, 0xc>(y);  // row_bcast:31 into rows 2 and 3
    return y;
}

// Sum over the wavefront's 64 lanes, the same bits in every lane (the last
// lane of the DPP scan, read as a scalar).
__device__ __forceinline__ float wave_sum(float y) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_incl_scan(y)), 63));
}

// Largest value over the wavefront and the lowest lane index holding it
// (index, not value, order on ties), by a DPP max-scan of (value, index)
// pairs; the same result in every lane.
__device__ __forceinline__ void wave_argmax(float &v, int &i) {
#define ARGMAX_STEP(CTRL, RM)                                   \
    {                                                          \
        const float ov = dpp_take_or<CTRL, RM>(v, -INFINITY);  \
        const int oi = dpp_take_or_i<CTRL, RM>(i, 0x7fffffff); \
        if (ov > v || (ov == v && oi < i)) {                   \
            v = ov;                                            \
            i = oi;                                            \
        }                                                      \
    }
    ARGMAX_STEP(0x111, 0xf)
    ARGMAX_STEP(0x112, 0xf)
    ARGMAX_STEP(0x114, 0xf)
    ARGMAX_STEP(0x118, 0xf)
    ARGMAX_STEP(0x142, 0xa)
    ARGMAX_STEP(0x143, 0xc)
#undef ARGMAX_STEP
    v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
    i = __builtin_amdgcn_readlane(i, 63);
}

__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_take_or<0x111, 0xf>(v, -INFINITY));
    v = fmaxf(v, dpp_take_or<0x112, 0xf>(v, -INFINITY));
    v = fmaxf(v, dpp_take_or<0x114, 0xf>(v, -INFINITY));
    v = fmaxf(v, dpp_take_or<0x118, 0xf>(v, -INFINITY));
    v = fmaxf(v, dpp_take_or<0x142, 0xa>(v, -INFINITY));
    v = fmaxf(v, dpp_take_or<0x143, 0xc>(v, -INFINITY));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }

// T log(1 + e^{x/T}) = LSE_T(0, x); 0 at x = -inf.
__device__ __forceinline__ float softplus_t(float x, const TParams &P) {
    if (x == -INFINITY) return 0.0f;
    float pos = x > 0.0f ? x : 0.0f;
    return pos + P.T * log1pf(expf(-fabsf(x) * P.invT));
}
// T log(e^{a/T} - 1) for a >= 0; -inf at a = 0.
__device__ __forceinline__ float lem_t(float a, const TParams &P) {
    if (!(a > 0.0f)) return -INFINITY;
    return a + P.T * logf(-expm1f(-a * P.invT));
}

// Message rows of two states hold one value, d = m1 - m0, in their first
// row (the second row of the slot is never read or written).  Every row is
// stored normalised, its larger state exactly zero (x - x = +0), so the two
// states come back exactly: m0 = -max(d, 0), m1 = min(d, 0).  Binary
// messages then move half the bytes.
__device__ __forceinline__ float pk_m0(float d) { return d > 0.0f ? -d : 0.0f; }
__device__ __forceinline__ float pk_m1(float d) { return d < 0.0f ? d : 0.0f; }
// states s0 .. s0 + N - 1 of the message row at p, a row of n states, into
// x (0 past the row's end, or everywhere when !ok, and then p is not read).
// MODE 2: the row is packed (n is 2, s0 is 0); MODE 1: packed when n is 2;
// MODE 0: one state per panel row whatever n (the reverse sweep's sums).
// Callers pick the mode once per tile or variable where they can, so the
// loads of an unrolled loop stay in one block.
template <int N, int MODE, class PT>
__device__ __forceinline__ void msg_load(PT p, int n, int s0, bool ok, float (&x)[N]) {
    static_assert(N >= 2, "a packed row yields two states");
    if (MODE == 2 || (MODE == 1 && n == 2)) {
        const float d = ok ? p[0] : 0.0f;
        x[0] = pk_m0(d);
        x[1] = pk_m1(d);
#pragma unroll
        for (int s = 2; s < N; ++s) x[s] = 0.0f;
        return;
    }
#pragma unroll
    for (int s = 0; s < N; ++s) x[s] = (ok && s0 + s < n) ? p[(s0 + s) * kLanes] : 0.0f;
}

// state s of the message row at p, a row of n states (packed when n == 2)
template <class PT>
__device__ __forceinline__ float msg_state(PT p, int n, int s) {
    if (n == 2) {
        const float d = p[0];
        return s == 0 ? pk_m0(d) : pk_m1(d);
    }
    return p[s * kLanes];
}

// damp, normalise and store one message row of n states held in registers
template <int N>
__device__ __forceinline__ void damp_store(float *row, const float (&mo)[N], const float (&u)[N], int n,
                                           const TParams &P) {
    float mn[N];
    float mx = -INFINITY;
#pragma unroll
    for (int s = 0; s < N; ++s)
        if (s < n) {
            float a = P.d * mo[s];
            float b = P.omd * u[s];
            mn[s] = a + b;
            mx = fmaxf(mx, mn[s]);
        }
    if (n == 2) {  // one of the two normalised states is +0, so the difference is exact
        row[0] = (mn[1 % N] - mx) - (mn[0] - mx);
        return;
    }
#pragma unroll
    for (int s = 0; s < N; ++s)
        if (s < n) row[s * kLanes] = mn[s] - mx;
}

// --------------------------------------------------------------------------
// variable phase
// --------------------------------------------------------------------------
// Three paths, chosen per variable by its degree and state count only:
//   low  (degree <= 16, <= 16 states): one lane per variable, tiles of 64
//   mid  (degree <= 64): one wavefront per variable, one edge per lane
//   high (larger degree): one 256-thread block per variable
// One launch covers all three: blocks [0, ceil((n_low+n_mid)/4)) run four
// wavefront items each (low tiles first, then mid variables), the remaining
// blocks one high variable each.

// low: NB >= states of every lane; edge rows fetched KU at a time (addresses,
// then rows, all in flight) and added in edge order.  MODE as for msg_load.
template <int NB, int MODE, class GV>
__device__ __forceinline__ void belief_low_tile_m(const GV &G, int t, int lane) {
    constexpr int KU = NB <= 4 ? 8 : 4;
    const VTile vt = G.vtile[t];
    const int n = G.vns[t * kLanes + lane];
    const int base = vt.b_off + lane;
    float acc[NB];
#pragma unroll
    for (int s = 0; s < NB; ++s) acc[s] = (s < n) ? G.theta[base + s * kLanes] : 0.0f;
    const int32_t *ea = G.vedge + vt.e_off + lane;
    for (int k0 = 0; k0 < vt.kmax; k0 += KU) {
        int a[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) a[u] = (k0 + u < vt.kmax) ? ea[(k0 + u) * kLanes] : -1;
        float x[KU][NB];
#pragma unroll
        for (int u = 0; u < KU; ++u) msg_load<NB, MODE>(G.m + (a[u] >= 0 ? a[u] : 0), n, 0, a[u] >= 0, x[u]);
#pragma unroll
        for (int u = 0; u < KU; ++u)
#pragma unroll
            for (int s = 0; s < NB; ++s)
                if (a[u] >= 0 && s < n) acc[s] += x[u][s];
    }
#pragma unroll
    for (int s = 0; s < NB; ++s)
        if (s < n) G.B[base + s * kLanes] = acc[s];
}

// A tile whose panel has two rows holds only two-state variables (and idle
// lanes): every row it reads is packed.
template <int NB, class GV>
__device__ __forceinline__ void belief_low_tile(const GV &G, int t, int lane) {
    if (G.raw_msgs) belief_low_tile_m<NB, 0>(G, t, lane);
    else if (G.vtile[t].n == 2) belief_low_tile_m<NB, 2>(G, t, lane);
    else belief_low_tile_m<NB, 1>(G, t, lane);
}

// The beliefs of two lane-path variables at once (va with na states, vb with
// nb) in registers, each with belief_low_tile's additions in its order (theta
// first, then the edges in order); both gathers are in flight together.
template <int NA, int NB, class GV>
__device__ __forceinline__ void belief_regs2(const GV &G, int va, int na, int vb, int nb, float (&ba)[NA],
                                             float (&bb)[NB]) {
    constexpr int KU = 4;
#pragma unroll
    for (int s = 0; s < NA; ++s) ba[s] = 0.0f;
#pragma unroll
    for (int s = 0; s < NB; ++s) bb[s] = 0.0f;
    const int ka = va >= 0 ? G.vtile[va >> 6].kmax : 0;
    const int kb = vb >= 0 ? G.vtile[vb >> 6].kmax : 0;
    const int32_t *ea = nullptr, *eb = nullptr;
    if (va >= 0) {
        const VTile vt = G.vtile[va >> 6];
        const int base = vt.b_off + (va & (kLanes - 1));
#pragma unroll
        for (int s = 0; s < NA; ++s)
            if (s < na) ba[s] = G.theta[base + s * kLanes];
        ea = G.vedge + vt.e_off + (va & (kLanes - 1));
    }
    if (vb >= 0) {
        const VTile vt = G.vtile[vb >> 6];
        const int base = vt.b_off + (vb & (kLanes - 1));
#pragma unroll
        for (int s = 0; s < NB; ++s)
            if (s < nb) bb[s] = G.theta[base + s * kLanes];
        eb = G.vedge + vt.e_off + (vb & (kLanes - 1));
    }
    const int kmax = ka > kb ? ka : kb;
    for (int k0 = 0; k0 < kmax; k0 += KU) {
        int a[KU], b[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            a[u] = (k0 + u < ka) ? ea[(k0 + u) * kLanes] : -1;
            b[u] = (k0 + u < kb) ? eb[(k0 + u) * kLanes] : -1;
        }
        float x[KU][NA], y[KU][NB];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            msg_load<NA, 1>(G.m + (a[u] >= 0 ? a[u] : 0), na, 0, a[u] >= 0, x[u]);
            msg_load<NB, 1>(G.m + (b[u] >= 0 ? b[u] : 0), nb, 0, b[u] >= 0, y[u]);
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
#pragma unroll
            for (int s = 0; s < NA; ++s)
                if (a[u] >= 0 && s < na) ba[s] += x[u][s];
#pragma unroll
            for (int s = 0; s < NB; ++s)
                if (b[u] >= 0 && s < nb) bb[s] += y[u][s];
        }
    }
}

// mid: lane l holds edge l; a wavefront sum (wave_sum: the same bits in
// every lane) adds up each state.
template <class GV>
__device__ __forceinline__ void belief_mid_var(const GV &G, int hv, int lane) {
    constexpr int SC = 8;
    const HVar h = G.hvar[hv];
    const int k = h.e_begin + lane;
    const int a = k < h.e_end ? G.hedge[k] : -1;
    for (int s0 = 0; s0 < h.n; s0 += SC) {
        // lane j's evidence term, loaded with the edge rows rather than
        // after the sums
        const bool own = lane < SC && s0 + lane < h.n;
        const float th = own ? G.theta[h.b_addr + (s0 + lane) * kLanes] : 0.0f;
        float x[SC];
        if (G.raw_msgs) msg_load<SC, 0>(G.m + (a >= 0 ? a : 0), h.n, s0, a >= 0, x);
        else msg_load<SC, 1>(G.m + (a >= 0 ? a : 0), h.n, s0, a >= 0, x);
#pragma unroll
        for (int j = 0; j < SC; ++j)
            if (s0 + j < h.n) x[j] = wave_sum(x[j]);  // uniform condition
        if (own) {
            float v = 0.0f;
#pragma unroll
            for (int j = 0; j < SC; ++j)
                if (j == lane) v = x[j];
            G.B[h.b_addr + (s0 + lane) * kLanes] = th + v;
        }
    }
}

// high: thread i sums edges i, i+256, ... in order (fetched 4 at a time);
// each wavefront combines its 64 partial sums (wave_sum), and the four
// wavefront sums are added in order.
constexpr int kHighThreads = 256;
constexpr int kHighWaves = kHighThreads / 64;
template <int MODE, class GV>
__device__ __forceinline__ void belief_high_var(const GV &G, int hv, int tid, float (*red)[kHighWaves]) {
    constexpr int SC = 8;  // states per pass
    constexpr int KC = 4;  // edges per thread fetched together
    const HVar h = G.hvar[hv];
    const int lane = tid & 63, wave = tid >> 6;
    for (int s0 = 0; s0 < h.n; s0 += SC) {
        const int ns = min(SC, h.n - s0);  // uniform
        // thread tid's evidence term, loaded with the edge rows rather than
        // after the reduction
        const float th = tid < ns ? G.theta[h.b_addr + (s0 + tid) * kLanes] : 0.0f;
        float part[SC];
#pragma unroll
        for (int j = 0; j < SC; ++j) part[j] = 0.0f;
        for (int k0 = h.e_begin + tid; k0 < h.e_end; k0 += KC * kHighThreads) {
            int a[KC];
#pragma unroll
            for (int u = 0; u < KC; ++u) {
                const int k = k0 + u * kHighThreads;
                a[u] = k < h.e_end ? G.hedge[k] : -1;
            }
            float x[KC][SC];
#pragma unroll
            for (int u = 0; u < KC; ++u)
                msg_load<SC, MODE>(G.m + (a[u] >= 0 ? a[u] : 0), h.n, s0, a[u] >= 0, x[u]);
#pragma unroll
            for (int u = 0; u < KC; ++u)
#pragma unroll
                for (int j = 0; j < SC; ++j)
                    if (a[u] >= 0 && j < ns) part[j] += x[u][j];
        }
#pragma unroll
        for (int j = 0; j < SC; ++j)
            if (j < ns) {
                part[j] = wave_sum(part[j]);
                if (lane == 0) red[j][wave] = part[j];
            }
        __syncthreads();
        if (tid < ns) {
            float v = red[tid][0];
#pragma unroll
            for (int w = 1; w < kHighWaves; ++w) v += red[tid][w];
            G.B[h.b_addr + (s0 + tid) * kLanes] = th + v;
        }
        __syncthreads();
    }
}

// column group (HVar.lanes = w > 1): variables l = 0..w-1 at belief
// addresses b_addr + l, edge rows [k][w].  Thread (kg, l), kg = tid / w,
// sums variable l's edges kg, kg + KG, ... (KG = 256 / w) in order, so each
// load instruction reads 64 / w runs of w adjacent messages.  The KG
// partial sums of a (variable, state) are then added in a fixed order: an
// xor tree over the 64 / w lanes of each wavefront that hold the variable,
// then the four wavefront sums in order.
constexpr int kColStates = 2;  // states per pass
constexpr int kColRound = 16;  // edges per thread fetched together
constexpr int kColRed = kColStates * kHighWaves * kColLanesMax;
template <int MODE, class GV>
__device__ __forceinline__ void belief_col_group(const GV &G, const HVar &h, int tid, float *red) {
    const int lsh = __builtin_ctz((unsigned)h.lanes), w = h.lanes;  // a power of two
    const int l = tid & (w - 1), kg = tid >> lsh, KG = kHighThreads >> lsh;
    const int kmax = (h.e_end - h.e_begin) >> lsh;
    for (int s0 = 0; s0 < h.n; s0 += kColStates) {
        const int ns = min(kColStates, h.n - s0);  // uniform
        // thread tid < w * ns writes variable tid % w, state s0 + tid / w;
        // its evidence term is loaded with the edge rows
        const bool own = tid < w * ns;
        const int ol = tid & (w - 1), os = s0 + (tid >> lsh);
        const float th = own ? G.theta[h.b_addr + ol + os * kLanes] : 0.0f;
        float part[kColStates];
#pragma unroll
        for (int j = 0; j < kColStates; ++j) part[j] = 0.0f;
        for (int k0 = kg; k0 < kmax; k0 += kColRound * KG) {
            int a[kColRound];
#pragma unroll
            for (int u = 0; u < kColRound; ++u) {
                const int k = k0 + u * KG;
                a[u] = k < kmax ? G.hedge[h.e_begin + (k << lsh) + l] : -1;
            }
            float x[kColRound][kColStates];
#pragma unroll
            for (int u = 0; u < kColRound; ++u)
                msg_load<kColStates, MODE>(G.m + (a[u] >= 0 ? a[u] : 0), h.n, s0, a[u] >= 0, x[u]);
#pragma unroll
            for (int u = 0; u < kColRound; ++u)
#pragma unroll
                for (int j = 0; j < kColStates; ++j)
                    if (a[u] >= 0 && j < ns) part[j] += x[u][j];
        }
        const int wave = tid >> 6;
#pragma unroll
        for (int j = 0; j < kColStates; ++j) {
            for (int msk = w; msk < kLanes; msk <<= 1) part[j] += __shfl_xor(part[j], msk);
            if ((tid & 63) < w) red[(j * kHighWaves + wave) * kColLanesMax + l] = part[j];
        }
        __syncthreads();
        if (own) {
            const float *r = red + (os - s0) * kHighWaves * kColLanesMax + ol;
            float v = r[0];
#pragma unroll
            for (int wv = 1; wv < kHighWaves; ++wv) v += r[wv * kColLanesMax];
            G.B[h.b_addr + ol + os * kLanes] = th + v;
        }
        __syncthreads();
    }
}

template <int NB>
__global__ __launch_bounds__(256) void k_belief(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                                int n_low, int n_mid, int n_high, int swz) {
    __shared__ float red[8][kHighWaves];
    __shared__ float cred[kColRed];
    // block-per-variable items first: they are the longest, so they start
    // before the wavefront items fill the machine
    if ((int)blockIdx.x < n_high) {
        const int hb = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
        const WorkItem it = items[n_low + n_mid + hb];
        const auto G = glob(gs[it.g]);
        const HVar h = G.hvar[it.t];
        // two-state rows are packed except in the reverse sweep's sums;
        // rows of other variables hold one state per panel row
        const bool pk = h.n == 2 && !G.raw_msgs;
        if (h.lanes > 1) {
            if (pk) belief_col_group<2>(G, h, threadIdx.x, cred);
            else belief_col_group<0>(G, h, threadIdx.x, cred);
        } else {
            if (pk) belief_high_var<2>(G, it.t, threadIdx.x, red);
            else belief_high_var<0>(G, it.t, threadIdx.x, red);
        }
        return;
    }
    const int nwave = n_low + n_mid;
    const int wave_blocks = (nwave + 3) / 4;
    const int bx = (int)blockIdx.x - n_high;
    const int b = swz ? swizzle_block(bx, wave_blocks) : bx;
    const int w = __builtin_amdgcn_readfirstlane(b * 4 + (int)(threadIdx.x >> 6));
    if (w >= nwave) return;
    const WorkItem it = items[w];
    if (w < n_low) belief_low_tile<NB>(glob(gs[it.g]), it.t, lane_id());
    else belief_mid_var(glob(gs[it.g]), it.t, lane_id());
}

// --------------------------------------------------------------------------
// factor phase: dense pairwise enumeration factors (one lane per factor)
// --------------------------------------------------------------------------
// u0[i] = LSE_T,j (phi(i,j) + n1[j]),  u1[j] = LSE_T,i (phi(i,j) + n0[i]);
// equal to LSE over the configurations with that slot fixed, minus the slot's
// own incoming term.  EXACT: NA x NB known at compile time; otherwise the
// tile's (a, b) <= (NA, NB) are read at run time with the same arithmetic.
// FUSED: the two slot beliefs are recomputed here from the messages being
// read (belief_regs2: the variable phase's additions in its order, both
// gathers in flight together) instead of being read from B, so one launch
// does a whole iteration; messages are then read from G.m and written to
// G.mo, a different buffer.  EARLY (fused only): the table is loaded before
// the belief gathers rather than after them, so more loads are in flight per
// wavefront at the cost of registers (fewer wavefronts per SIMD): faster when
// the graph streams from HBM, slower when it sits in the last-level cache.
// The arithmetic is the same either way.
template <int NA, int NB, bool EXACT, bool MAXP, bool FUSED, bool EARLY = false, class GV>
__device__ __forceinline__ void pair_tile(const GV &G, const FTile &ft, int lane, const TParams &P, int t = -1) {
    const int na = EXACT ? NA : ft.a;
    const int nb = EXACT ? NB : ft.b;
    const float *r0 = G.m + ft.m_off + lane;
    const float *r1 = r0 + na * kLanes;
    float *w0 = G.mo + ft.m_off + lane;
    float *w1 = w0 + na * kLanes;
    const float *ph = G.phi + ft.phi_off + lane;
    float p[NA][NB];
    auto load_table = [&]() {
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (i < na && j < nb) p[i][j] = ph[(i * nb + j) * kLanes];
    };
    if (EARLY) load_table();
    float m0[NA], m1[NB], x0[NA], x1[NB];
    if (FUSED) {
        float b0[NA], b1[NB];
        // slot variables: from the tile's slot bases where the lanes hold
        // consecutive variables (uniform), else one index per lane
        const int a0 = t >= 0 ? G.faff[2 * t] : -1, a1 = t >= 0 ? G.faff[2 * t + 1] : -1;
        const int va = a0 >= 0 ? (lane < ft.nact ? a0 + lane : -1) : G.fvar[ft.vb_off + lane];
        const int vb = a1 >= 0 ? (lane < ft.nact ? a1 + lane : -1) : G.fvar[ft.vb_off + kLanes + lane];
        belief_regs2<NA, NB>(G, va, na, vb, nb, b0, b1);
        msg_load<NA, 1>(r0, na, 0, true, m0);
        msg_load<NB, 1>(r1, nb, 0, true, m1);
#pragma unroll
        for (int i = 0; i < NA; ++i)
            if (i < na) x0[i] = b0[i] - m0[i];
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < nb) x1[j] = b1[j] - m1[j];
    } else {
        const int va = G.fvb[ft.vb_off + lane];
        const int vb = G.fvb[ft.vb_off + kLanes + lane];
        msg_load<NA, 1>(r0, na, 0, true, m0);
        msg_load<NB, 1>(r1, nb, 0, true, m1);
#pragma unroll
        for (int i = 0; i < NA; ++i)
            if (i < na) x0[i] = G.B[va + i * kLanes] - m0[i];
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < nb) x1[j] = G.B[vb + j * kLanes] - m1[j];
    }
    if (!EARLY) load_table();
    float u0[NA], u1[NB];
    // to slot 0
#pragma unroll
    for (int i = 0; i < NA; ++i)
        if (i < na) {
            float t[NB];
            float M = -INFINITY;
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j < nb) {
                    t[j] = p[i][j] + x1[j];
                    M = fmaxf(M, t[j]);
                }
            if (MAXP) {
                u0[i] = M;
            } else {
                float s = 0.0f;
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    if (j < nb) s += fexp2((t[j] - M) * P.c);
                u0[i] = M + flog2(s) * P.r;
            }
        }
    // to slot 1
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < nb) {
            float t[NA];
            float M = -INFINITY;
#pragma unroll
            for (int i = 0; i < NA; ++i)
                if (i < na) {
                    t[i] = p[i][j] + x0[i];
                    M = fmaxf(M, t[i]);
                }
            if (MAXP) {
                u1[j] = M;
            } else {
                float s = 0.0f;
#pragma unroll
                for (int i = 0; i < NA; ++i)
                    if (i < na) s += fexp2((t[i] - M) * P.c);
                u1[j] = M + flog2(s) * P.r;
            }
        }
    damp_store<NA>(w0, m0, u0, na, P);
    damp_store<NB>(w1, m1, u1, nb, P);
}

template <int NA, int NB, bool EXACT, bool MAXP, bool FUSED, bool EARLY>
__global__ __launch_bounds__(256) void k_pair(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                              int nitems, TParams P, int swz) {
    const int w = wave_item(swz);
    if (w >= nitems) return;
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    const FTile ft = G.ftile[it.t];
    pair_tile<NA, NB, EXACT, MAXP, FUSED, EARLY>(G, ft, lane_id(), P, it.t);
}

// Square pairwise tiles of several state counts (2..8) in one launch: each
// wavefront branches on its tile's state count (uniform across the
// wavefront) to that count's exact tile code, so a tile gets the same bits as
// in its own class's launch.
template <bool MAXP, bool FUSED, bool EARLY>
__global__ __launch_bounds__(256) void k_pair_mix(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                                  int nitems, TParams P, int swz) {
    const int w = wave_item(swz);
    if (w >= nitems) return;
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    const FTile ft = G.ftile[it.t];
    const int lane = lane_id();
    switch (__builtin_amdgcn_readfirstlane(ft.a)) {
    case 2: pair_tile<2, 2, true, MAXP, FUSED, EARLY>(G, ft, lane, P, it.t); break;
    case 3: pair_tile<3, 3, true, MAXP, FUSED, EARLY>(G, ft, lane, P, it.t); break;
    case 4: pair_tile<4, 4, true, MAXP, FUSED, EARLY>(G, ft, lane, P, it.t); break;
    case 5: pair_tile<5, 5, true, MAXP, FUSED, EARLY>(G, ft, lane, P, it.t); break;
    case 6: pair_tile<6, 6, true, MAXP, FUSED, EARLY>(G, ft, lane, P, it.t); break;
    case 7: pair_tile<7, 7, true, MAXP, FUSED, EARLY>(G, ft, lane, P, it.t); break;
    default: pair_tile<8, 8, true, MAXP, FUSED, EARLY>(G, ft, lane, P, it.t); break;
    }
}

// --------------------------------------------------------------------------
// factor phase: OR / AND, closed forms (PGMax Sec. "Package features":
// logical factors with updates linear in their arity)
// --------------------------------------------------------------------------
// With delta_j = n[j,1] - n[j,0] (negated for AND, De Morgan), parents j < p,
// child p:
//   T = 0: S_-i = sum_{j != i} relu(delta_j), M_-i = max_{j != i} delta_j
//          child  u = (0, S + min(0, max_j delta_j))
//          parent u = (max(0, delta_c + S_-i + min(0, M_-i)), delta_c + S_-i)
//   T > 0: A_-i = sum_{j != i} sp_T(delta_j)
//          child  u = (0, lem_T(A))
//          parent u = (sp_T(delta_c + lem_T(A_-i)), delta_c + A_-i)
// The leave-one-out sums are exclusive prefix + suffix sums, never total minus
// own term.  For AND the two entries of u are swapped.

// one lane per factor, at most kLogLaneArityMax edges
template <bool MAXP, class GV>
__device__ __forceinline__ void logl_tile(const GV &G, const FTile &ft, int lane, const TParams &P) {
    constexpr int K = kLogLaneArityMax;
    const int k = ft.a, p = k - 1;
    const bool flip = ft.b != 0;
    const float *rows = G.m + ft.m_off + lane;
    float *wrows = G.mo + ft.m_off + lane;
    float m0[K], m1[K], dl[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j < k) {
            const float dj = rows[(2 * j) * kLanes];  // packed binary row
            m0[j] = pk_m0(dj);
            m1[j] = pk_m1(dj);
            const int vb = G.fvb[ft.vb_off + j * kLanes + lane];
            const float n0 = G.B[vb] - m0[j];
            const float n1 = G.B[vb + kLanes] - m1[j];
            dl[j] = flip ? (n0 - n1) : (n1 - n0);
        }
    float dc = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j == p) dc = dl[j];
    float t[K], pre[K], suf[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j < p) t[j] = MAXP ? fmaxf(dl[j], 0.0f) : softplus_t(dl[j], P);
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j < p) {
            pre[j] = acc;
            acc += t[j];
        }
    const float total = acc;
    acc = 0.0f;
#pragma unroll
    for (int j = K - 1; j >= 0; --j)
        if (j < p) {
            suf[j] = acc;
            acc += t[j];
        }
    float max1 = -INFINITY, max2 = -INFINITY;
    int amax = 0;
    if (MAXP) {
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < p && dl[j] > max1) {
                max1 = dl[j];
                amax = j;
            }
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < p && j != amax) max2 = fmaxf(max2, dl[j]);
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j < k) {
            float a0, a1;
            if (j == p) {
                a0 = 0.0f;
                a1 = MAXP ? total + fminf(0.0f, max1) : lem_t(total, P);
            } else {
                const float loo = pre[j] + suf[j];
                a1 = dc + loo;
                if (MAXP) {
                    const float mo = (j == amax) ? max2 : max1;
                    a0 = fmaxf(0.0f, dc + loo + fminf(0.0f, mo));
                } else {
                    a0 = softplus_t(dc + lem_t(loo, P), P);
                }
            }
            const float u0 = flip ? a1 : a0, u1 = flip ? a0 : a1;
            const float w0 = P.d * m0[j] + P.omd * u0, w1 = P.d * m1[j] + P.omd * u1;
            const float mx = fmaxf(w0, w1);
            wrows[(2 * j) * kLanes] = (w1 - mx) - (w0 - mx);
        }
}

// one wavefront per factor; edge j sits in chunk j/64 at lane j%64
template <int CH, bool MAXP, class GV>
__device__ __forceinline__ void logw_tile(const GV &G, const FTile &ft, int lane, const TParams &P) {
    const int k = ft.a, p = k - 1;
    const int nch = (k + kLanes - 1) / kLanes;
    const bool flip = ft.b != 0;
    float m0[CH], m1[CH], dl[CH], t[CH], pre[CH], suf[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int j = c * kLanes + lane;
        dl[c] = 0.0f;
        t[c] = 0.0f;
        if (c < nch && j < k) {
            const float dm = G.m[ft.m_off + c * 2 * kLanes + lane];  // packed binary row
            m0[c] = pk_m0(dm);
            m1[c] = pk_m1(dm);
            const int vb = G.fvb[ft.vb_off + j];
            const float n0 = G.B[vb] - m0[c];
            const float n1 = G.B[vb + kLanes] - m1[c];
            dl[c] = flip ? (n0 - n1) : (n1 - n0);
            if (j < p) t[c] = MAXP ? fmaxf(dl[c], 0.0f) : softplus_t(dl[c], P);
        }
    }
    // child delta
    float dc = 0.0f;
#pragma unroll
    for (int c = 0; c < CH; ++c)
        if (c == p / kLanes) dc = __shfl(dl[c], p % kLanes, 64);
    // exclusive prefix sums over parents, chunk-major (DPP scans)
    float carry = 0.0f;
#pragma unroll
    for (int c = 0; c < CH; ++c)
        if (c < nch) {
            const float x = wave_incl_scan(t[c]);
            float ex = __shfl_up(x, 1, 64);
            if (lane == 0) ex = 0.0f;
            pre[c] = carry + ex;
            carry += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
        }
    const float total = carry;
    // exclusive suffix sums: the same scan over the lanes in reverse order
    carry = 0.0f;
#pragma unroll
    for (int c = CH - 1; c >= 0; --c)
        if (c < nch) {
            const float x = wave_incl_scan(__shfl(t[c], 63 - lane, 64));  // lane l: sum of t[63-l..63]
            float ex = __shfl(x, 62 - lane, 64);                          // sum of t[l+1..63]
            if (lane == 63) ex = 0.0f;
            suf[c] = carry + ex;
            carry += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
        }
    float max1 = -INFINITY, max2 = -INFINITY;
    int amax = 0x7fffffff;
    if (MAXP) {
        // largest parent delta, lowest index on ties
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int j = c * kLanes + lane;
            if (c < nch && j < p && (dl[c] > max1 || (dl[c] == max1 && j < amax))) {
                max1 = dl[c];
                amax = j;
            }
        }
        wave_argmax(max1, amax);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int j = c * kLanes + lane;
            if (c < nch && j < p && j != amax) max2 = fmaxf(max2, dl[c]);
        }
        max2 = wave_max(max2);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int j = c * kLanes + lane;
        if (c < nch && j < k) {
            float a0, a1;
            if (j == p) {
                a0 = 0.0f;
                a1 = MAXP ? total + fminf(0.0f, max1) : lem_t(total, P);
            } else {
                const float loo = pre[c] + suf[c];
                a1 = dc + loo;
                if (MAXP) {
                    const float mo = (j == amax) ? max2 : max1;
                    a0 = fmaxf(0.0f, dc + loo + fminf(0.0f, mo));
                } else {
                    a0 = softplus_t(dc + lem_t(loo, P), P);
                }
            }
            const float u0 = flip ? a1 : a0, u1 = flip ? a0 : a1;
            const float w0 = P.d * m0[c] + P.omd * u0, w1 = P.d * m1[c] + P.omd * u1;
            const float mx = fmaxf(w0, w1);
            G.mo[ft.m_off + c * 2 * kLanes + lane] = (w1 - mx) - (w0 - mx);
        }
    }
}

// All logical tiles of at most 4 chunks (256 edges) in one launch: a
// wavefront runs a lane-per-factor tile or one wide factor.
template <bool MAXP>
__global__ __launch_bounds__(256) void k_logical(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                                 int nitems, TParams P, int swz) {
    const int w = wave_item(swz);
    if (w >= nitems) return;
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    const FTile ft = G.ftile[it.t];
    if (ft.kind == TK_LOGL) logl_tile<MAXP>(G, ft, lane_id(), P);
    else logw_tile<4, MAXP>(G, ft, lane_id(), P);
}

// logical factors of 257 .. 1024 edges
template <bool MAXP>
__global__ __launch_bounds__(256) void k_logical_wide(const DevGraph *__restrict__ gs,
                                                      const WorkItem *__restrict__ items, int nitems, TParams P,
                                                      int swz) {
    const int w = wave_item(swz);
    if (w >= nitems) return;
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    logw_tile<kLogWaveChunks, MAXP>(G, G.ftile[it.t], lane_id(), P);
}

// --------------------------------------------------------------------------
// resident solver: a small graph in one workgroup
// --------------------------------------------------------------------------
// The graph's messages and beliefs are copied into LDS; each iteration runs
// the variable launches' items and then the factor launches' items, one
// wavefront per item with the launched path's tile code, the two phases
// separated by workgroup barriers.  The tile code reads and writes through a
// copy of the graph descriptor whose message and belief arrays are the LDS
// copies, so every element gets the same arithmetic as in launched
// iterations; the messages are copied back at the end.
constexpr int kSolveThreads = 512;

template <bool MAXP, class GV>
__device__ __forceinline__ void pair_any(const GV &G, const FTile &ft, int lane, const TParams &P) {
    if (ft.a == ft.b) switch (ft.a) {
        case 2: pair_tile<2, 2, true, MAXP, false, false>(G, ft, lane, P); return;
        case 3: pair_tile<3, 3, true, MAXP, false, false>(G, ft, lane, P); return;
        case 4: pair_tile<4, 4, true, MAXP, false, false>(G, ft, lane, P); return;
        case 5: pair_tile<5, 5, true, MAXP, false, false>(G, ft, lane, P); return;
        case 6: pair_tile<6, 6, true, MAXP, false, false>(G, ft, lane, P); return;
        case 7: pair_tile<7, 7, true, MAXP, false, false>(G, ft, lane, P); return;
        case 8: pair_tile<8, 8, true, MAXP, false, false>(G, ft, lane, P); return;
        default: break;
        }
    pair_tile<kPairStatesMax, kPairStatesMax, false, MAXP, false, false>(G, ft, lane, P);
}

// Address of graph array `a` in G (as 4-byte words).
__device__ __forceinline__ const uint32_t *solve_src(const DevGraph &G, int a) {
    switch (a) {
    case SA_M: return (const uint32_t *)G.m;
    case SA_B: return (const uint32_t *)G.B;
    case SA_VEDGE: return (const uint32_t *)G.vedge;
    case SA_FVB: return (const uint32_t *)G.fvb;
    case SA_HEDGE: return (const uint32_t *)G.hedge;
    case SA_VNS: return (const uint32_t *)G.vns;
    case SA_VTILE: return (const uint32_t *)G.vtile;
    case SA_FTILE: return (const uint32_t *)G.ftile;
    case SA_HVAR: return (const uint32_t *)G.hvar;
    case SA_THETA: return (const uint32_t *)G.theta;
    default: return (const uint32_t *)G.phi;
    }
}

__device__ __forceinline__ void solve_repoint(DevGraph &G, int a, uint32_t *p) {
    switch (a) {
    case SA_M: G.m = (float *)p; G.mo = (float *)p; break;
    case SA_B: G.B = (float *)p; break;
    case SA_VEDGE: G.vedge = (const int32_t *)p; break;
    case SA_FVB: G.fvb = (const int32_t *)p; break;
    case SA_HEDGE: G.hedge = (const int32_t *)p; break;
    case SA_VNS: G.vns = (const int32_t *)p; break;
    case SA_VTILE: G.vtile = (const VTile *)p; break;
    case SA_FTILE: G.ftile = (const FTile *)p; break;
    case SA_HVAR: G.hvar = (const HVar *)p; break;
    case SA_THETA: G.theta = (float *)p; break;
    default: G.phi = (float *)p; break;
    }
}

template <bool MAXP>
__global__ __launch_bounds__(kSolveThreads) void k_solve_resident(const DevGraph *__restrict__ gs, SolvePlan plan,
                                                                  int iters, TParams P) {
    extern __shared__ __align__(16) uint32_t lds[];
    const DevGraph &Gg = gs[0];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kSolveThreads / 64;
    DevGraph G = Gg;
    uint32_t *at = lds;
#pragma unroll
    for (int a = 0; a < SA_COUNT; ++a) {  // unrolled: each field chosen at compile time
        if (!(plan.lds_mask >> a & 1u)) continue;
        const uint32_t *src = solve_src(Gg, a);
        for (int i = tid; i < plan.words[a]; i += kSolveThreads) at[i] = src[i];
        solve_repoint(G, a, at);
        at += solve_words_aligned(plan.words[a]);
    }
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        for (int li = 0; li < plan.nv; ++li) {
            const SolveLaunch L = plan.l[li];
            for (int w = wave; w < L.n + L.n_mid; w += nwaves) {
                const int t = L.items[w].t;
                if (w >= L.n) {
                    belief_mid_var(G, t, lane);
                    continue;
                }
                switch (L.a) {
                case 2: belief_low_tile<2>(G, t, lane); break;
                case 4: belief_low_tile<4>(G, t, lane); break;
                case 8: belief_low_tile<8>(G, t, lane); break;
                default: belief_low_tile<16>(G, t, lane); break;
                }
            }
        }
        __syncthreads();
        for (int li = plan.nv; li < plan.nv + plan.nf; ++li) {
            const SolveLaunch L = plan.l[li];
            for (int w = wave; w < L.n; w += nwaves) {
                const FTile ft = G.ftile[L.items[w].t];
                if (L.kind == TK_PAIR) pair_any<MAXP>(G, ft, lane, P);
                else if (ft.kind == TK_LOGL) logl_tile<MAXP>(G, ft, lane, P);
                else logw_tile<4, MAXP>(G, ft, lane, P);
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < plan.words[SA_M]; i += kSolveThreads) Gg.m[i] = G.m[i];
}

// --------------------------------------------------------------------------
// factor phase: generic enumeration factors (explicit configuration tables or
// dense tables of arity != 2 / larger state counts).  One wavefront per
// block, one lane per factor; the class's configuration table is staged in
// LDS, incoming terms and per-(slot,state) accumulators live in LDS.
// u[e_j,s] = LSE_T{score(c) : c_j = s} - n[e_j,s],  score(c) = phi(c) + sum_l n[e_l,c_l]
// --------------------------------------------------------------------------
// One tile of a generic class: `rows` holds the class's configuration rows
// (C x A bytes), nv / acc / sacc are [R][64] float arrays in LDS.
template <bool MAXP, class GV>
__device__ __forceinline__ void gen_tile(const GV &G, const FTile &ft, int lane, const TParams &P,
                                         uint8_t *rows, float *nv, float *acc, float *sacc) {
    const GenClass gc = G.gcls[ft.a];
    const int A = gc.arity, C = gc.ncfg;
    for (int i = lane; i < C * A; i += kLanes) rows[i] = G.grows[gc.rows_off + i];
    const float *mrow = G.m + ft.m_off + lane;
    float *wrow = G.mo + ft.m_off + lane;
    for (int j = 0; j < A; ++j) {
        const int vb = G.fvb[ft.vb_off + j * kLanes + lane];
        for (int s = 0; s < gc.slot_n[j]; ++s) {
            const int r = gc.slot_row[j] + s;
            nv[r * kLanes + lane] = G.B[vb + s * kLanes] - msg_state(mrow + gc.slot_row[j] * kLanes, gc.slot_n[j], s);
            acc[r * kLanes + lane] = -INFINITY;
            sacc[r * kLanes + lane] = 0.0f;
        }
    }
    __syncthreads();
    const float *ph = G.phi + ft.phi_off + lane;
    for (int c = 0; c < C; ++c) {
        float sc = ph[c * kLanes];
        for (int j = 0; j < A; ++j) sc += nv[rows[c * A + j] * kLanes + lane];
        for (int j = 0; j < A; ++j) {
            const int r = rows[c * A + j];
            acc[r * kLanes + lane] = fmaxf(acc[r * kLanes + lane], sc);
        }
    }
    if (!MAXP) {
        for (int c = 0; c < C; ++c) {
            float sc = ph[c * kLanes];
            for (int j = 0; j < A; ++j) sc += nv[rows[c * A + j] * kLanes + lane];
            for (int j = 0; j < A; ++j) {
                const int r = rows[c * A + j];
                sacc[r * kLanes + lane] += fexp2((sc - acc[r * kLanes + lane]) * P.c);
            }
        }
    }
    for (int j = 0; j < A; ++j) {
        const int r0 = gc.slot_row[j], n = gc.slot_n[j];
        float mx = -INFINITY;
        for (int s = 0; s < n; ++s) {
            const int r = r0 + s;
            const float lse =
                MAXP ? acc[r * kLanes + lane] : acc[r * kLanes + lane] + flog2(sacc[r * kLanes + lane]) * P.r;
            const float u = lse - nv[r * kLanes + lane];
            const float mn = P.d * msg_state(mrow + r0 * kLanes, n, s) + P.omd * u;
            sacc[r * kLanes + lane] = mn;  // reuse as staging for the normalisation
            mx = fmaxf(mx, mn);
        }
        if (n == 2) {  // packed: one of the two normalised states is +0
            wrow[r0 * kLanes] = (sacc[(r0 + 1) * kLanes + lane] - mx) - (sacc[r0 * kLanes + lane] - mx);
            continue;
        }
        for (int s = 0; s < n; ++s) {
            const int r = r0 + s;
            wrow[r * kLanes] = sacc[r * kLanes + lane] - mx;
        }
    }
}

// Dense three-way classes with N states in every slot (N^3 <= 64
// configurations, last slot fastest): one lane per factor with the table,
// incoming terms and scores in registers.  The generic class layout (rows of
// slot j at j*N), so the reverse sweep's generic kernel serves these tiles.
// u_j[s] = LSE_T{score(c) : c_j = s} - n_j[s], score = phi + n_0 + n_1 + n_2.
template <int N, bool MAXP, class GV>
__device__ __forceinline__ void tri_tile(const GV &G, const FTile &ft, int lane, const TParams &P) {
    const float *mrow = G.m + ft.m_off + lane;
    float m[3][N], x[3][N];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int vb = G.fvb[ft.vb_off + j * kLanes + lane];
#pragma unroll
        for (int s = 0; s < N; ++s) {
            m[j][s] = msg_state(mrow + j * N * kLanes, N, s);
            x[j][s] = G.B[vb + s * kLanes] - m[j][s];
        }
    }
    const float *ph = G.phi + ft.phi_off + lane;
    float sc[N][N][N];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int c = 0; c < N; ++c) sc[a][b][c] = ph[((a * N + b) * N + c) * kLanes] + x[0][a] + x[1][b] + x[2][c];
    float u[3][N];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int s = 0; s < N; ++s) {
            float M = -INFINITY;
#pragma unroll
            for (int p = 0; p < N; ++p)
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    const float v = j == 0 ? sc[s][p][q] : j == 1 ? sc[p][s][q] : sc[p][q][s];
                    M = fmaxf(M, v);
                }
            if (MAXP) {
                u[j][s] = M - x[j][s];
            } else {
                float e = 0.0f;
#pragma unroll
                for (int p = 0; p < N; ++p)
#pragma unroll
                    for (int q = 0; q < N; ++q) {
                        const float v = j == 0 ? sc[s][p][q] : j == 1 ? sc[p][s][q] : sc[p][q][s];
                        e += fexp2((v - M) * P.c);
                    }
                u[j][s] = M + flog2(e) * P.r - x[j][s];
            }
        }
    float *wrow = G.mo + ft.m_off + lane;
#pragma unroll
    for (int j = 0; j < 3; ++j) damp_store<N>(wrow + j * N * kLanes, m[j], u[j], N, P);
}

template <int N, bool MAXP>
__global__ __launch_bounds__(256) void k_tri(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                             int nitems, TParams P) {
    const int w = wave_index(4);
    if (w >= nitems) return;
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    tri_tile<N, MAXP>(G, G.ftile[it.t], lane_id(), P);
}

// Any class within the kernel limits: LDS for the largest (80 KB), which
// leaves room for two such blocks per CU.
template <bool MAXP>
__global__ __launch_bounds__(64) void k_gen(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                            int nitems, TParams P) {
    __shared__ uint8_t rows[kGenCfgMax * kGenArityMax];
    __shared__ float nv[kGenRowsMax * kLanes];
    __shared__ float acc[kGenRowsMax * kLanes];
    __shared__ float sacc[kGenRowsMax * kLanes];
    const int w = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
    if (w >= nitems) return;
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    gen_tile<MAXP>(G, G.ftile[it.t], lane_id(), P, rows, nv, acc, sacc);
}

// Classes whose rows and accumulators fit the launch's dynamic LDS (sized
// per launch group from its classes), so many blocks share a CU.
template <bool MAXP>
__global__ __launch_bounds__(64) void k_gen_dyn(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                                int nitems, TParams P, int rows_bytes, int nrows) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
    if (w >= nitems) return;
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    float *nv = (float *)(smem + rows_bytes);
    float *acc = nv + nrows * kLanes;
    float *sacc = acc + nrows * kLanes;
    gen_tile<MAXP>(G, G.ftile[it.t], lane_id(), P, smem, nv, acc, sacc);
}

// --------------------------------------------------------------------------
// adjoint of the unrolled damped sum-product iterations (T > 0)
// --------------------------------------------------------------------------
// Reverse mode of one iteration t (m_t -> m_{t+1}).  The adjoint of m_{t+1}
// is held in two parts, A[e,s] + Bbar[var(e),s]: A is the direct part owned
// by the factor of e, Bbar the adjoint of the next iterate's beliefs.  Per
// factor, with u, m' = d m + (1-d) u recomputed from m_t:
//   gm  = A + Bbar[var]                         adjoint of m_{t+1}
//   gmp = gm - [s = argmax m'] sum_s gm         normalisation m_{t+1} = m' - max m'
//   gu  = (1-d) gmp
//   sbar(c) = sum_j gu[e_j,c_j] pi_j(c),  pi_j(c) = exp((score(c) - LSE_j,c_j)/T)
//   phibar(c) += sbar(c)
//   nbar[e_j,s] = sum_{c: c_j = s} sbar(c) - gu[e_j,s]
//   A <- d gmp - nbar                           direct part of the adjoint of m_t
// The variable side (Bbar_t = sum_e nbar, thetabar += Bbar_t) runs the belief
// kernels on nbar.
template <int NA, int NB, bool EXACT>
__global__ __launch_bounds__(256) void k_pair_adj(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                                  int nitems, TParams P, AdjBufs J) {
    const int w = wave_index(4);
    if (w >= nitems) return;
    const int lane = lane_id();
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    const FTile ft = G.ftile[it.t];
    const int na = EXACT ? NA : ft.a;
    const int nb = EXACT ? NB : ft.b;
    const int va = G.fvb[ft.vb_off + lane];
    const int vb = G.fvb[ft.vb_off + kLanes + lane];
    const int o0 = ft.m_off + lane, o1 = o0 + na * kLanes;
    float m0[NA], m1[NB], x0[NA], x1[NB];
    msg_load<NA, 1>(G.m + o0, na, 0, true, m0);
    msg_load<NB, 1>(G.m + o1, nb, 0, true, m1);
#pragma unroll
    for (int i = 0; i < NA; ++i)
        if (i < na) x0[i] = G.B[va + i * kLanes] - m0[i];
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < nb) x1[j] = G.B[vb + j * kLanes] - m1[j];
    const float *ph = G.phi + ft.phi_off + lane;
    float p[NA][NB];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (i < na && j < nb) p[i][j] = ph[(i * nb + j) * kLanes];
    // forward: u (LSE per row / column), exactly as in the forward kernel
    float u0[NA], u1[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i)
        if (i < na) {
            float t[NB];
            float M = -INFINITY;
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j < nb) {
                    t[j] = p[i][j] + x1[j];
                    M = fmaxf(M, t[j]);
                }
            float sm = 0.0f;
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j < nb) sm += fexp2((t[j] - M) * P.c);
            u0[i] = M + flog2(sm) * P.r;
        }
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < nb) {
            float t[NA];
            float M = -INFINITY;
#pragma unroll
            for (int i = 0; i < NA; ++i)
                if (i < na) {
                    t[i] = p[i][j] + x0[i];
                    M = fmaxf(M, t[i]);
                }
            float sm = 0.0f;
#pragma unroll
            for (int i = 0; i < NA; ++i)
                if (i < na) sm += fexp2((t[i] - M) * P.c);
            u1[j] = M + flog2(sm) * P.r;
        }
    // adjoint of damping + normalisation
    float gu0[NA], gu1[NB], dg0[NA], dg1[NB];
    {
        float mx = -INFINITY, tot = 0.0f, gm[NA];
        int am = 0;
#pragma unroll
        for (int i = 0; i < NA; ++i)
            if (i < na) {
                const float mp = P.d * m0[i] + P.omd * u0[i];
                if (mp > mx) {
                    mx = mp;
                    am = i;
                }
                gm[i] = J.A[o0 + i * kLanes] + J.Bbar[va + i * kLanes];
                tot += gm[i];
            }
#pragma unroll
        for (int i = 0; i < NA; ++i)
            if (i < na) {
                const float gmp = gm[i] - (i == am ? tot : 0.0f);
                gu0[i] = P.omd * gmp;
                dg0[i] = P.d * gmp;
            }
    }
    {
        float mx = -INFINITY, tot = 0.0f, gm[NB];
        int am = 0;
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < nb) {
                const float mp = P.d * m1[j] + P.omd * u1[j];
                if (mp > mx) {
                    mx = mp;
                    am = j;
                }
                gm[j] = J.A[o1 + j * kLanes] + J.Bbar[vb + j * kLanes];
                tot += gm[j];
            }
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < nb) {
                const float gmp = gm[j] - (j == am ? tot : 0.0f);
                gu1[j] = P.omd * gmp;
                dg1[j] = P.d * gmp;
            }
    }
    // configuration adjoints
    float rs0[NA], rs1[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i) rs0[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < NB; ++j) rs1[j] = 0.0f;
    float *pb = J.phibar + ft.phi_off + lane;
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (i < na && j < nb) {
                const float pa = fexp2((p[i][j] + x1[j] - u0[i]) * P.c);
                const float pbv = fexp2((p[i][j] + x0[i] - u1[j]) * P.c);
                const float sb = gu0[i] * pa + gu1[j] * pbv;
                pb[(i * nb + j) * kLanes] += sb;
                rs0[i] += sb;
                rs1[j] += sb;
            }
#pragma unroll
    for (int i = 0; i < NA; ++i)
        if (i < na) {
            const float nbar = rs0[i] - gu0[i];
            J.nbar[o0 + i * kLanes] = nbar;
            J.A[o0 + i * kLanes] = dg0[i] - nbar;
        }
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < nb) {
            const float nbar = rs1[j] - gu1[j];
            J.nbar[o1 + j * kLanes] = nbar;
            J.A[o1 + j * kLanes] = dg1[j] - nbar;
        }
}

// generic enumeration factors (one wavefront per block, LDS as in k_gen)
__global__ __launch_bounds__(64) void k_gen_adj(const DevGraph *__restrict__ gs, const WorkItem *__restrict__ items,
                                                int nitems, TParams P, AdjBufs J) {
    __shared__ uint8_t rows[kGenCfgMax * kGenArityMax];
    __shared__ float nv[kGenRowsMax][kLanes];
    __shared__ float lse[kGenRowsMax][kLanes];
    __shared__ float acc[kGenRowsMax][kLanes];
    __shared__ float gu[kGenRowsMax][kLanes];
    __shared__ float dg[kGenRowsMax][kLanes];
    const int w = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
    if (w >= nitems) return;
    const int lane = lane_id();
    const WorkItem it = items[w];
    const GGraph G = glob(gs[it.g]);
    const FTile ft = G.ftile[it.t];
    const GenClass gc = G.gcls[ft.a];
    const int A = gc.arity, C = gc.ncfg;
    for (int i = lane; i < C * A; i += kLanes) rows[i] = G.grows[gc.rows_off + i];
    const int base = ft.m_off + lane;
    for (int j = 0; j < A; ++j) {
        const int vb = G.fvb[ft.vb_off + j * kLanes + lane];
        for (int s = 0; s < gc.slot_n[j]; ++s) {
            const int r = gc.slot_row[j] + s;
            nv[r][lane] = G.B[vb + s * kLanes] - msg_state(G.m + base + gc.slot_row[j] * kLanes, gc.slot_n[j], s);
            lse[r][lane] = -INFINITY;
            acc[r][lane] = 0.0f;
        }
    }
    __syncthreads();
    const float *ph = G.phi + ft.phi_off + lane;
    for (int c = 0; c < C; ++c) {
        float sc = ph[c * kLanes];
        for (int j = 0; j < A; ++j) sc += nv[rows[c * A + j]][lane];
        for (int j = 0; j < A; ++j) {
            const int r = rows[c * A + j];
            lse[r][lane] = fmaxf(lse[r][lane], sc);
        }
    }
    for (int c = 0; c < C; ++c) {
        float sc = ph[c * kLanes];
        for (int j = 0; j < A; ++j) sc += nv[rows[c * A + j]][lane];
        for (int j = 0; j < A; ++j) {
            const int r = rows[c * A + j];
            acc[r][lane] += fexp2((sc - lse[r][lane]) * P.c);
        }
    }
    for (int j = 0; j < A; ++j) {
        const int vb = G.fvb[ft.vb_off + j * kLanes + lane];
        const int r0 = gc.slot_row[j], n = gc.slot_n[j];
        float mx = -INFINITY, tot = 0.0f;
        int am = 0;
        for (int s = 0; s < n; ++s) {
            const int r = r0 + s;
            lse[r][lane] = lse[r][lane] + flog2(acc[r][lane]) * P.r;
            const float u = lse[r][lane] - nv[r][lane];
            const float mp = P.d * msg_state(G.m + base + r0 * kLanes, n, s) + P.omd * u;
            if (mp > mx) {
                mx = mp;
                am = s;
            }
            const float gm = J.A[base + r * kLanes] + J.Bbar[vb + s * kLanes];
            gu[r][lane] = gm;
            tot += gm;
        }
        for (int s = 0; s < n; ++s) {
            const int r = r0 + s;
            const float gmp = gu[r][lane] - (s == am ? tot : 0.0f);
            gu[r][lane] = P.omd * gmp;
            dg[r][lane] = P.d * gmp;
            acc[r][lane] = 0.0f;
        }
    }
    float *pb = J.phibar + ft.phi_off + lane;
    for (int c = 0; c < C; ++c) {
        float sc = ph[c * kLanes];
        for (int j = 0; j < A; ++j) sc += nv[rows[c * A + j]][lane];
        float sb = 0.0f;
        for (int j = 0; j < A; ++j) {
            const int r = rows[c * A + j];
            sb += gu[r][lane] * fexp2((sc - lse[r][lane]) * P.c);
        }
        pb[c * kLanes] += sb;
        for (int j = 0; j < A; ++j) acc[rows[c * A + j]][lane] += sb;
    }
    for (int r = 0; r < gc.nrows; ++r) {
        const float nbar = acc[r][lane] - gu[r][lane];
        J.nbar[base + r * kLanes] = nbar;
        J.A[base + r * kLanes] = dg[r][lane] - nbar;
    }
}

// Adjoint of the read-out q = B - LSE_T(B): Bbar = gq - softmax(B/T) sum gq;
// it is also the first contribution to thetabar.
__global__ __launch_bounds__(256) void k_readout_adj(const DevGraph *__restrict__ gs, int ntiles, TParams P,
                                                     const float *__restrict__ gq, float *__restrict__ bbar,
                                                     float *__restrict__ thetabar) {
    const int w = wave_index(4);
    if (w >= ntiles) return;
    const int lane = lane_id();
    const GGraph G = glob(gs[0]);
    const int v = w * kLanes + lane;
    if (v >= G.V) return;
    const int n = G.vn[v];
    const int b0 = G.vtile[w].b_off + lane;
    const float *b = G.B + b0;
    const float *g = gq + G.vs_off[v];
    float M = -INFINITY, tot = 0.0f;
    for (int s = 0; s < n; ++s) {
        M = fmaxf(M, b[s * kLanes]);
        tot += g[s];
    }
    float z = 0.0f;
    for (int s = 0; s < n; ++s) z += fexp2((b[s * kLanes] - M) * P.c);
    const float iz = 1.0f / z;
    for (int s = 0; s < n; ++s) {
        const float pr = fexp2((b[s * kLanes] - M) * P.c) * iz;
        const float x = g[s] - pr * tot;
        bbar[b0 + s * kLanes] = x;
        thetabar[b0 + s * kLanes] = x;
    }
}

__global__ void k_accumulate(float *__restrict__ y, const float *__restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += x[i];
}

__global__ void k_logpot_out(const DevGraph *__restrict__ gs, const float *__restrict__ panel, float *__restrict__ out) {
    const GGraph G = glob(gs[0]);
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= G.F) return;
    const int base = G.fac_phi[f];
    if (base < 0) return;
    const int64_t o = G.lp_off[f];
    const int n = (int)(G.lp_off[f + 1] - o);
    for (int c = 0; c < n; ++c) out[o + c] = panel[base + c * kLanes];
}

__global__ void k_evidence_out(const DevGraph *__restrict__ gs, const float *__restrict__ panel,
                               float *__restrict__ out) {
    const GGraph G = glob(gs[0]);
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= G.V) return;
    const float *row = panel + G.vtile[v / kLanes].b_off + (v % kLanes);
    const int64_t o = G.vs_off[v];
    for (int s = 0; s < G.vn[v]; ++s) out[o + s] = row[s * kLanes];
}

// --------------------------------------------------------------------------
// read-out and flat-order exchange
// --------------------------------------------------------------------------
// q[v,s] = B[v,s] - LSE_T(B[v,:]) (or B), MAP = lowest-index argmax.
// Variable tile w of G; flag_host (may be null) is also set on a non-finite
// belief.
template <bool MAXP, class GV>
__device__ __forceinline__ void readout_tile(const GV &G, int w, const TParams &P, float *__restrict__ qout,
                                             int normalized, int32_t *__restrict__ mapout,
                                             int32_t *__restrict__ flag_host) {
    const int lane = lane_id();
    const int v = w * kLanes + lane;
    if (v >= G.V) return;
    const VTile vt = G.vtile[w];
    const int n = G.vn[v];
    const float *b = G.B + vt.b_off + lane;
    float M = -INFINITY;
    int best = 0;
    bool finite = true;
    for (int s = 0; s < n; ++s) {
        const float x = b[s * kLanes];
        finite = finite && isfinite(x);
        if (x > M) {
            M = x;
            best = s;
        }
    }
    if (!finite) {
        G.flag[0] = 1;
        if (flag_host) flag_host[0] = 1;
    }
    if (mapout) mapout[G.vext ? G.vext[v] : v] = best;
    if (qout) {
        float z = 0.0f;
        if (normalized) {
            if (MAXP) {
                z = M;
            } else {
                float s = 0.0f;
                for (int t = 0; t < n; ++t) s += fexp2((b[t * kLanes] - M) * P.c);
                z = M + flog2(s) * P.r;
            }
        }
        float *q = qout + G.vs_off[v];
        for (int s = 0; s < n; ++s) q[s] = b[s * kLanes] - z;
    }
}

template <bool MAXP>
__global__ __launch_bounds__(256) void k_readout(const DevGraph *__restrict__ gs, int ntiles, TParams P,
                                                 float *__restrict__ qout, int normalized,
                                                 int32_t *__restrict__ mapout) {
    const int w = wave_index(4);
    if (w >= ntiles) return;
    readout_tile<MAXP>(glob(gs[0]), w, P, qout, normalized, mapout, nullptr);
}

// Read-outs of several graphs in one launch: blockIdx.y = job, each job's
// normalised beliefs and MAP written straight to its (page-locked host)
// outputs, and its flag word set on a non-finite belief.
__global__ __launch_bounds__(256) void k_readout_multi(const ReadJob *__restrict__ jobs) {
    const ReadJob J = jobs[blockIdx.y];
    const int w = wave_index(4);
    if (w >= J.ntiles) return;
    if (J.maxp) readout_tile<true>(glob(*J.g), w, J.P, J.q, 1, J.map, J.flag);
    else readout_tile<false>(glob(*J.g), w, J.P, J.q, 1, J.map, J.flag);
}

__global__ void k_msgs_out(const DevGraph *__restrict__ gs, float *__restrict__ out) {
    const GGraph G = glob(gs[0]);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= G.E) return;
    const float *row = G.m + G.edge_maddr[e];
    const int64_t o = G.es_off[e];
    const int n = (int)(G.es_off[e + 1] - o);
    for (int s = 0; s < n; ++s) out[o + s] = msg_state(row, n, s);
}

__global__ void k_msgs_in(const DevGraph *__restrict__ gs, const float *__restrict__ in) {
    const GGraph G = glob(gs[0]);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= G.E) return;
    float *row = G.m + G.edge_maddr[e];
    const int64_t o = G.es_off[e];
    const int n = (int)(G.es_off[e + 1] - o);
    if (n == 2) {  // packed: the row is normalised first (its larger state to +0)
        const float v0 = in[o], v1 = in[o + 1], mx = fmaxf(v0, v1);
        row[0] = (v1 - mx) - (v0 - mx);
        return;
    }
    for (int s = 0; s < n; ++s) row[s * kLanes] = in[o + s];
}

__global__ void k_evidence_in(const DevGraph *__restrict__ gs, const float *__restrict__ in) {
    const GGraph G = glob(gs[0]);
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= G.V) return;
    float *row = G.theta + G.vtile[v / kLanes].b_off + (v % kLanes);
    const int64_t o = G.vs_off[v];
    for (int s = 0; s < G.vn[v]; ++s) row[s * kLanes] = in[o + s];
}

// Residual of an iteration: the largest |m - mprev| over the edge-state
// entries (flat mapping; padding lanes excluded), per block, NaN and
// infinity as infinity; then one block takes the maximum of the block
// results.  Maxima do not depend on the order of reduction.
constexpr int kResidualThreads = 256;
__host__ __device__ inline int residual_block_count(int E) {
    return ((E > 1 ? E : 1) + kResidualThreads - 1) / kResidualThreads;
}

template <class GV>
__device__ __forceinline__ void residual_partial(const GV &G, const float *__restrict__ mprev,
                                                 float *__restrict__ partial, int block, float (&red)[256]) {
    const int e = block * kResidualThreads + (int)threadIdx.x;
    float r = 0.0f;
    if (e < G.E) {
        const int a = G.edge_maddr[e];
        const int n = (int)(G.es_off[e + 1] - G.es_off[e]);
        for (int s = 0; s < n; ++s) {
            const float d = fabsf(msg_state(G.m + a, n, s) - msg_state(mprev + a, n, s));
            r = (d == d && d <= 3.0e38f) ? fmaxf(r, d) : INFINITY;
        }
    }
    red[threadIdx.x] = r;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[block] = red[0];
}

__device__ __forceinline__ void max_final(const float *__restrict__ partial, int n, float *__restrict__ out,
                                          float (&red)[256]) {
    float r = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) r = fmaxf(r, partial[i]);
    red[threadIdx.x] = r;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(256) void k_residual(const DevGraph *__restrict__ gs, const float *__restrict__ mprev,
                                                  float *__restrict__ partial) {
    __shared__ float red[256];
    residual_partial(glob(gs[0]), mprev, partial, (int)blockIdx.x, red);
}

__global__ __launch_bounds__(256) void k_max_final(const float *__restrict__ partial, int n, float *__restrict__ out) {
    __shared__ float red[256];
    max_final(partial, n, out, red);
}

// The same checks for several graphs at once (one per blockIdx.y, resp.
// blockIdx.x): the copy of the messages taken before an iteration, then the
// residual of that iteration into out[slot].
__global__ __launch_bounds__(256) void k_save_multi(const ConvJob *__restrict__ jobs) {
    const ConvJob J = jobs[blockIdx.y];
    const float4 *src = reinterpret_cast<const float4 *>(J.g->m);
    float4 *dst = reinterpret_cast<float4 *>(J.mprev);
    for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < J.M / 4; i += (int)(gridDim.x * blockDim.x))
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_residual_multi(const ConvJob *__restrict__ jobs) {
    __shared__ float red[256];
    const ConvJob J = jobs[blockIdx.y];
    if ((int)blockIdx.x >= residual_block_count(J.E)) return;  // uniform over the block
    residual_partial(glob(*J.g), J.mprev, J.partial, (int)blockIdx.x, red);
}

__global__ __launch_bounds__(256) void k_max_final_multi(const ConvJob *__restrict__ jobs, float *__restrict__ out) {
    __shared__ float red[256];
    const ConvJob J = jobs[blockIdx.x];
    max_final(J.partial, residual_block_count(J.E), out + J.slot, red);
}

// Evidence panel of sample blockIdx.y = base panel + that sample's noise
// (flat variable-state order), in FP32.
__global__ void k_evidence_perturb(const DevGraph *__restrict__ views, const float *__restrict__ base,
                                   const float *__restrict__ noise, int64_t VS) {
    const int s = blockIdx.y;
    const GGraph G = glob(views[s]);
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= G.V) return;
    const int64_t addr = G.vtile[v / kLanes].b_off + (v % kLanes);
    const float *nz = noise + (int64_t)s * VS + G.vs_off[v];
    for (int t = 0; t < G.vn[v]; ++t) G.theta[addr + t * kLanes] = base[addr + t * kLanes] + nz[t];
}

__global__ void k_logpot_in(const DevGraph *__restrict__ gs, const float *__restrict__ in) {
    const GGraph G = glob(gs[0]);
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= G.F) return;
    const int base = G.fac_phi[f];
    if (base < 0) return;
    const int64_t o = G.lp_off[f];
    const int n = (int)(G.lp_off[f + 1] - o);
    for (int c = 0; c < n; ++c) G.phi[base + c * kLanes] = in[o + c];
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ----------------------------------------------------------------- launchers
hipError_t launch_belief(const DevGraph *gs, const WorkItem *items, int n_low, int n_mid, int n_high, int bucket,
                         const LaunchShape &S, hipStream_t st) {
    if (n_low + n_mid + n_high <= 0) return hipSuccess;
    dim3 grid(blocks_for(n_low + n_mid, 4) + n_high), block(256);
    const int z = S.swizzle;
    switch (bucket) {
    case 2: hipLaunchKernelGGL((k_belief<2>), grid, block, 0, st, gs, items, n_low, n_mid, n_high, z); break;
    case 4: hipLaunchKernelGGL((k_belief<4>), grid, block, 0, st, gs, items, n_low, n_mid, n_high, z); break;
    case 8: hipLaunchKernelGGL((k_belief<8>), grid, block, 0, st, gs, items, n_low, n_mid, n_high, z); break;
    default: hipLaunchKernelGGL((k_belief<16>), grid, block, 0, st, gs, items, n_low, n_mid, n_high, z); break;
    }
    return hipGetLastError();
}

template <bool MAXP, bool FUSED, bool EARLY>
static void pair_dispatch(const DevGraph *gs, const WorkItem *items, int n, int na, int nb, const TParams &P,
                          const LaunchShape &S, hipStream_t st) {
    dim3 grid(blocks_for(n, S.wpb)), block(64 * S.wpb);
    const int z = S.swizzle;
#define PAIR_CASE(N)                                                                                          \
    case N:                                                                                                   \
        hipLaunchKernelGGL((k_pair<N, N, true, MAXP, FUSED, EARLY>), grid, block, 0, st, gs, items, n, P, z); \
        return;
    if (na == nb) {
        switch (na) {
            PAIR_CASE(2)
            PAIR_CASE(3)
            PAIR_CASE(4)
            PAIR_CASE(5)
            PAIR_CASE(6)
            PAIR_CASE(7)
            PAIR_CASE(8)
        default: break;
        }
    }
#undef PAIR_CASE
    if (na == 0) {
        hipLaunchKernelGGL((k_pair_mix<MAXP, FUSED, EARLY>), grid, block, 0, st, gs, items, n, P, z);
        return;
    }
    if (!FUSED)
        hipLaunchKernelGGL((k_pair<kPairStatesMax, kPairStatesMax, false, MAXP, false, false>), grid, block, 0, st,
                           gs, items, n, P, z);
}

hipError_t launch_pair(const DevGraph *gs, const WorkItem *items, int n, int na, int nb, bool maxp,
                       const TParams &P, const LaunchShape &S, hipStream_t st, bool fused) {
    if (n <= 0) return hipSuccess;
    // na = nb = 0: a mixed launch of square tiles of 2..kPairStatesMax states
    if (na != nb && (na == 0 || nb == 0)) return hipErrorInvalidValue;
    if (fused && na != 0 && (na != nb || na < 2 || na > kPairStatesMax)) return hipErrorInvalidValue;
    if (fused && S.early) {
        if (maxp) pair_dispatch<true, true, true>(gs, items, n, na, nb, P, S, st);
        else pair_dispatch<false, true, true>(gs, items, n, na, nb, P, S, st);
    } else if (fused) {
        if (maxp) pair_dispatch<true, true, false>(gs, items, n, na, nb, P, S, st);
        else pair_dispatch<false, true, false>(gs, items, n, na, nb, P, S, st);
    } else {
        if (maxp) pair_dispatch<true, false, false>(gs, items, n, na, nb, P, S, st);
        else pair_dispatch<false, false, false>(gs, items, n, na, nb, P, S, st);
    }
    return hipGetLastError();
}

int32_t solve_lds_limit(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return v;
}

hipError_t launch_solve_resident(const DevGraph *g, const SolvePlan &plan, int32_t iters, bool maxp, const TParams &P,
                                 hipStream_t st) {
    if (iters <= 0) return hipSuccess;
    const uint32_t need = (1u << SA_M) | (1u << SA_B);
    int64_t words = 0;
    for (int a = 0; a < SA_COUNT; ++a)
        if (plan.lds_mask >> a & 1u) words += solve_words_aligned(plan.words[a]);
    if ((plan.lds_mask & need) != need || plan.lds_mask >> SA_COUNT || words != plan.lds_words || plan.nv < 0 ||
        plan.nf < 0 || plan.nv + plan.nf > kSolveLaunchesMax)
        return hipErrorInvalidValue;
    for (int i = 0; i < plan.nv + plan.nf; ++i) {
        const SolveLaunch &L = plan.l[i];
        if (L.n < 0 || L.n_mid < 0 || (L.n + L.n_mid > 0 && !L.items)) return hipErrorInvalidValue;
        if (i < plan.nv ? L.kind != -1 : (L.kind != TK_PAIR && L.kind != TK_LOGL)) return hipErrorInvalidValue;
    }
    const size_t lds = sizeof(uint32_t) * (size_t)words;
    const void *fn = maxp ? (const void *)k_solve_resident<true> : (const void *)k_solve_resident<false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (maxp) hipLaunchKernelGGL((k_solve_resident<true>), dim3(1), dim3(kSolveThreads), lds, st, g, plan, iters, P);
    else hipLaunchKernelGGL((k_solve_resident<false>), dim3(1), dim3(kSolveThreads), lds, st, g, plan, iters, P);
    return hipGetLastError();
}

hipError_t launch_logical(const DevGraph *gs, const WorkItem *items, int n, bool wide, bool maxp, const TParams &P,
                          const LaunchShape &S, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    dim3 grid(blocks_for(n, S.wpb)), block(64 * S.wpb);
    const int z = S.swizzle;
    if (wide) {
        if (maxp) hipLaunchKernelGGL((k_logical_wide<true>), grid, block, 0, st, gs, items, n, P, z);
        else hipLaunchKernelGGL((k_logical_wide<false>), grid, block, 0, st, gs, items, n, P, z);
    } else {
        if (maxp) hipLaunchKernelGGL((k_logical<true>), grid, block, 0, st, gs, items, n, P, z);
        else hipLaunchKernelGGL((k_logical<false>), grid, block, 0, st, gs, items, n, P, z);
    }
    return hipGetLastError();
}

hipError_t launch_gen(const DevGraph *gs, const WorkItem *items, int n, bool maxp, const TParams &P, int lds_code,
                      hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (lds_code < 0) {  // dense three-way, -N states per slot
        dim3 grid(blocks_for(n, 4)), block(256);
        switch (-lds_code) {
#define TRI_CASE(K)                                                                                 \
    case K:                                                                                         \
        if (maxp) hipLaunchKernelGGL((k_tri<K, true>), grid, block, 0, st, gs, items, n, P);     \
        else hipLaunchKernelGGL((k_tri<K, false>), grid, block, 0, st, gs, items, n, P);         \
        break;
            TRI_CASE(2)
            TRI_CASE(3)
            TRI_CASE(4)
#undef TRI_CASE
        default: return hipErrorInvalidValue;
        }
    } else if (lds_code == 0) {
        if (maxp) hipLaunchKernelGGL((k_gen<true>), dim3(n), dim3(64), 0, st, gs, items, n, P);
        else hipLaunchKernelGGL((k_gen<false>), dim3(n), dim3(64), 0, st, gs, items, n, P);
    } else {
        int rows_bytes, nrows;
        gen_lds_decode(lds_code, &rows_bytes, &nrows);
        const size_t shm = (size_t)rows_bytes + (size_t)3 * nrows * kLanes * sizeof(float);
        if (maxp) hipLaunchKernelGGL((k_gen_dyn<true>), dim3(n), dim3(64), shm, st, gs, items, n, P, rows_bytes, nrows);
        else hipLaunchKernelGGL((k_gen_dyn<false>), dim3(n), dim3(64), shm, st, gs, items, n, P, rows_bytes, nrows);
    }
    return hipGetLastError();
}

hipError_t launch_readout(const DevGraph *gs, int nvtiles, bool maxp, const TParams &P, float *q, int normalized,
                          int32_t *map, hipStream_t st) {
    if (nvtiles <= 0) return hipSuccess;
    dim3 grid(blocks_for(nvtiles, 4)), block(256);
    if (maxp) hipLaunchKernelGGL((k_readout<true>), grid, block, 0, st, gs, nvtiles, P, q, normalized, map);
    else hipLaunchKernelGGL((k_readout<false>), grid, block, 0, st, gs, nvtiles, P, q, normalized, map);
    return hipGetLastError();
}

hipError_t launch_readout_multi(const ReadJob *jobs, int n, int max_tiles, hipStream_t st) {
    if (n <= 0 || max_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_readout_multi, dim3(blocks_for(max_tiles, 4), n), dim3(256), 0, st, jobs);
    return hipGetLastError();
}

hipError_t launch_msgs_out(const DevGraph *gs, int E, float *out, hipStream_t st) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_msgs_out, dim3(blocks_for(E, 256)), dim3(256), 0, st, gs, out);
    return hipGetLastError();
}

hipError_t launch_msgs_in(const DevGraph *gs, int E, const float *in, hipStream_t st) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_msgs_in, dim3(blocks_for(E, 256)), dim3(256), 0, st, gs, in);
    return hipGetLastError();
}

hipError_t launch_evidence_in(const DevGraph *gs, int V, const float *in, hipStream_t st) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_evidence_in, dim3(blocks_for(V, 256)), dim3(256), 0, st, gs, in);
    return hipGetLastError();
}

int residual_blocks(int E) { return residual_block_count(E); }

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_addr[kScratchDevices] = {};
}  // namespace

hipError_t noalloc_scratch_address(int device, float **out) {
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = static_cast<float *>(p);
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

hipError_t launch_residual(const DevGraph *gs, int E, const float *mprev, float *partial, float *out, hipStream_t st) {
    const int nb = residual_blocks(E);
    hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, st, gs, mprev, partial);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, st, partial, nb, out);
    return hipGetLastError();
}

// ------------------------------------------------------- bandwidth probes
// Plain streaming kernels that measure what an ordinary kernel reaches on
// this device: float4 accesses, grid-stride, four float4 per thread in flight
// per pass.  Every loaded component feeds the sum, and the sum is stored only
// when it equals a value that finite sums of the probe's zero-filled data
// never take, so no load can be dropped.
namespace {
constexpr float kProbeNever = -1.2345e-37f;

__global__ __launch_bounds__(256) void k_stream_read(const float4 *__restrict__ src, int64_t n4,
                                                     float *__restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.0f;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        acc += ((a.x + a.y) + (a.z + a.w)) + ((b.x + b.y) + (b.z + b.w)) + ((c.x + c.y) + (c.z + c.w)) +
               ((d.x + d.y) + (d.z + d.w));
    }
    for (; i < n4; i += stride) {
        const float4 a = src[i];
        acc += (a.x + a.y) + (a.z + a.w);
    }
    if (acc == kProbeNever) sink[0] = acc;
}

__global__ __launch_bounds__(256) void k_stream_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                     int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_stream_write(float4 *__restrict__ dst, int64_t n4, float v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const float4 x = make_float4(v, v, v, v);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) dst[i] = x;
}

// reads five float4 per float4 written (src: 5 * m float4, dst: m float4),
// about the read/write mix of an iteration's factor launches
__global__ __launch_bounds__(256) void k_stream_mix(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                    int64_t m) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        float4 a = src[i];
#pragma unroll
        for (int k = 1; k < 5; ++k) {
            const float4 b = src[i + k * m];
            a.x += b.x;
            a.y += b.y;
            a.z += b.z;
            a.w += b.w;
        }
        dst[i] = a;
    }
}
}  // namespace

hipError_t launch_stream_probe(int kind, const void *src, void *dst, int64_t bytes, int blocks, hipStream_t st) {
    const int64_t n4 = bytes / 16;
    switch (kind) {
    case 0:
        hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(256), 0, st, (const float4 *)src, n4, (float *)dst);
        break;
    case 1:
        hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, st, (const float4 *)src, (float4 *)dst, n4);
        break;
    case 2: hipLaunchKernelGGL(k_stream_write, dim3(blocks), dim3(256), 0, st, (float4 *)dst, n4, 0.0f); break;
    default:
        hipLaunchKernelGGL(k_stream_mix, dim3(blocks), dim3(256), 0, st, (const float4 *)src, (float4 *)dst,
                           n4 / 5);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_save_multi(const ConvJob *jobs, int n, int max_M, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned bx = std::min<unsigned>(blocks_for(std::max(max_M / 4, 1), 256), 1024);
    hipLaunchKernelGGL(k_save_multi, dim3(bx, n), dim3(256), 0, st, jobs);
    return hipGetLastError();
}

hipError_t launch_residual_multi(const ConvJob *jobs, int n, int max_E, float *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_residual_multi, dim3(residual_block_count(max_E), n), dim3(256), 0, st, jobs);
    hipLaunchKernelGGL(k_max_final_multi, dim3(n), dim3(256), 0, st, jobs, out);
    return hipGetLastError();
}

hipError_t launch_evidence_perturb(const DevGraph *views, int S, int V, const float *base, const float *noise,
                                  int64_t VS, hipStream_t st) {
    if (V <= 0 || S <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_evidence_perturb, dim3(blocks_for(V, 256), S), dim3(256), 0, st, views, base, noise, VS);
    return hipGetLastError();
}

hipError_t launch_logpot_in(const DevGraph *gs, int F, const float *in, hipStream_t st) {
    if (F <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_logpot_in, dim3(blocks_for(F, 256)), dim3(256), 0, st, gs, in);
    return hipGetLastError();
}

hipError_t launch_pair_adj(const DevGraph *gs, const WorkItem *items, int n, int na, int nb, const TParams &P,
                           const AdjBufs &J, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (na <= 0 || nb <= 0) return hipErrorInvalidValue;  // mixed launches are forward only
    dim3 grid(blocks_for(n, 4)), block(256);
    if (na == nb && na >= 2 && na <= 8) {
        switch (na) {
        case 2: hipLaunchKernelGGL((k_pair_adj<2, 2, true>), grid, block, 0, st, gs, items, n, P, J); break;
        case 3: hipLaunchKernelGGL((k_pair_adj<3, 3, true>), grid, block, 0, st, gs, items, n, P, J); break;
        case 4: hipLaunchKernelGGL((k_pair_adj<4, 4, true>), grid, block, 0, st, gs, items, n, P, J); break;
        case 5: hipLaunchKernelGGL((k_pair_adj<5, 5, true>), grid, block, 0, st, gs, items, n, P, J); break;
        case 6: hipLaunchKernelGGL((k_pair_adj<6, 6, true>), grid, block, 0, st, gs, items, n, P, J); break;
        case 7: hipLaunchKernelGGL((k_pair_adj<7, 7, true>), grid, block, 0, st, gs, items, n, P, J); break;
        default: hipLaunchKernelGGL((k_pair_adj<8, 8, true>), grid, block, 0, st, gs, items, n, P, J); break;
        }
    } else {
        hipLaunchKernelGGL((k_pair_adj<kPairStatesMax, kPairStatesMax, false>), grid, block, 0, st, gs, items, n, P, J);
    }
    return hipGetLastError();
}

hipError_t launch_gen_adj(const DevGraph *gs, const WorkItem *items, int n, const TParams &P, const AdjBufs &J,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_adj, dim3(n), dim3(64), 0, st, gs, items, n, P, J);
    return hipGetLastError();
}

hipError_t launch_readout_adj(const DevGraph *gs, int nvtiles, const TParams &P, const float *gq, float *bbar,
                              float *thetabar, hipStream_t st) {
    if (nvtiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_readout_adj, dim3(blocks_for(nvtiles, 4)), dim3(256), 0, st, gs, nvtiles, P, gq, bbar,
                       thetabar);
    return hipGetLastError();
}

hipError_t launch_accumulate(float *y, const float *x, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_accumulate, dim3(blocks_for(n, 256)), dim3(256), 0, st, y, x, n);
    return hipGetLastError();
}

hipError_t launch_logpot_out(const DevGraph *gs, int F, const float *panel, float *out, hipStream_t st) {
    if (F <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_logpot_out, dim3(blocks_for(F, 256)), dim3(256), 0, st, gs, panel, out);
    return hipGetLastError();
}

hipError_t launch_evidence_out(const DevGraph *gs, int V, const float *panel, float *out, hipStream_t st) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_evidence_out, dim3(blocks_for(V, 256)), dim3(256), 0, st, gs, panel, out);
    return hipGetLastError();
}

TParams make_params(float damping, float temperature) {
    TParams P;
    P.d = damping;
    P.omd = 1.0f - damping;
    P.T = temperature;
    if (temperature > 0.0f) {
        P.invT = 1.0f / temperature;
        P.c = (float)(1.4426950408889634 / (double)temperature);  // log2(e) / T
        P.r = (float)((double)temperature * 0.6931471805599453);  // T ln 2
    } else {
        P.invT = 0.0f;
        P.c = 0.0f;
        P.r = 0.0f;
    }
    return P;
}

}  // namespace lbp
