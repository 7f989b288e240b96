// Internal data layout of liblbp.so, shared by the host graph compiler, the
// C-ABI implementation and the HIP kernels.
//
// Every per-edge and per-variable array lives in 64-wide panels: a factor
// tile holds up to 64 factors of one shape class, and state s of an edge sits
// at  edge_addr + 64*s,  where edge_addr = panel_base + row*64 + lane.  One
// wavefront handles one tile with one factor per lane, so every load and
// store of messages, potentials, beliefs and evidence is a unit-stride
// 256-byte access.  Large logical factors take a whole wavefront each; their
// edges fill 64-lane chunks of the same panel form.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace lbp {

constexpr int kLanes = 64;
constexpr int kMaxStates = 64;        // states per variable
constexpr int kLowDegMax = 16;        // lane-per-variable belief path: at most this many edges
constexpr int kLowStatesMax = 16;     //   and at most this many states
constexpr int kMidDegMax = 64;        // wavefront-per-variable path up to this degree, block-per-variable above
constexpr int kPairStatesMax = 8;     // dense pairwise fast path, both slots
constexpr int kLogLaneArityMax = 8;   // OR/AND with at most this many edges: one lane per factor
constexpr int kLogWaveArityMax = 1024;  // larger OR/AND: one wavefront per factor
constexpr int kLogWaveChunks = kLogWaveArityMax / kLanes;
constexpr int kGenArityMax = 8;       // generic enumeration factors
constexpr int kGenCfgMax = 4096;
constexpr int kGenRowsMax = 64;       // summed slot states of a generic factor

enum TileKind : int32_t { TK_PAIR = 0, TK_LOGL = 1, TK_LOGW = 2, TK_GEN = 3 };

// One factor tile (one wavefront of work).
struct FTile {
    int32_t kind;
    int32_t a;        // PAIR: states of slot 0; LOGL/LOGW: arity; GEN: class index
    int32_t b;        // PAIR: states of slot 1; LOGL/LOGW: 1 for AND, 0 for OR
    int32_t nact;     // factors in the tile (LOGW: 1)
    int32_t m_off;    // message panel base
    int32_t phi_off;  // potential panel base (PAIR, GEN), 0 otherwise
    int32_t vb_off;   // base of the belief-address rows [slot or chunk][64]
    int32_t pad;
};

// One variable tile: 64 consecutive variables.
struct VTile {
    int32_t b_off;    // belief / evidence panel base
    int32_t n;        // panel rows (max states over the tile)
    int32_t kmax;     // edge-address rows for the low-degree lanes
    int32_t e_off;    // base of the edge-address rows [k][64]
};

// A variable handled by the wavefront- or block-per-variable belief path,
// or (block path, lanes > 1) a column group: `lanes` consecutive variables
// of one belief panel (belief addresses b_addr + l) with equal state counts,
// whose edge addresses form rows [k][lanes] in e_begin..e_end, -1 past a
// variable's last edge.  The compiler forms a group where the variables'
// k-th edges mostly sit side by side in the message panels (the hidden
// units of a dense bipartite layer), so one load reads a run of them.
constexpr int kColLanesMin = 4, kColLanesMax = 16;
struct HVar {
    int32_t b_addr;   // belief address of state 0
    int16_t n;        // states
    int16_t lanes;    // 1, or the column group's variables (4, 8 or 16)
    int32_t e_begin;  // range in the high-degree edge-address list
    int32_t e_end;
};

// Generic enumeration class: a configuration table and the state counts of
// its slots.  rows[c*arity + j] = slot_row[j] + state of slot j in config c.
struct GenClass {
    int32_t arity;
    int32_t ncfg;
    int32_t nrows;    // sum of slot state counts
    int32_t rows_off; // offset into the uint8 row table
    int32_t slot_n[kGenArityMax];
    int32_t slot_row[kGenArityMax];
};

// LDS of the generic-class kernel for a class of `cells` = configurations x
// arity row bytes and `nrows` summed slot states: rows rounded up to 256
// bytes, then three [nrows][64] float arrays.  Launch groups of generic
// classes are keyed by gen_lds_code (0 when the need exceeds kGenDynLdsMax,
// for the kernel with static LDS for the largest class).
constexpr int kGenDynLdsMax = 48 * 1024;
inline int gen_lds_code(int cells, int nrows) {
    const int rb = (cells + 255) / 256 * 256;
    const int need = rb + 3 * nrows * 64 * 4;
    return need <= kGenDynLdsMax ? (rb / 256) * 128 + nrows : 0;
}
inline void gen_lds_decode(int code, int *rows_bytes, int *nrows) {
    *rows_bytes = (code / 128) * 256;
    *nrows = code % 128;
}

// Device pointers of one uploaded graph.
struct DevGraph {
    float *m;             // messages (panels) + a zero panel at zero_addr
    float *mo;            // where factor kernels write updated messages (== m: in place)
    float *B;             // beliefs (panels)
    float *theta;         // evidence (panels)
    float *phi;           // potentials (panels)
    const FTile *ftile;
    const int32_t *fvb;   // belief address of each (tile, slot, lane)
    const int32_t *fvar;  // variable of each (tile, slot, lane), -1 for idle lanes
    const int32_t *faff;  // per pairwise tile and slot: v0 when lane l < nact holds variable v0 + l, else -1
    const VTile *vtile;
    const int32_t *vedge; // message address of each (var tile, k, lane)
    const int32_t *vns;   // states of each low-degree lane, 0 for others
    const HVar *hvar;
    const int32_t *hedge;
    const GenClass *gcls;
    const uint8_t *grows;
    // flat-order mapping (read-out, state exchange)
    const int32_t *edge_maddr;   // E
    const int64_t *es_off;       // E+1
    const int64_t *vs_off;       // V+1, by internal id: offset in the caller's flat order
    const int32_t *vn;           // V
    const int32_t *vext;         // V: the caller's id of each internal id, or null (same order)
    const int32_t *fac_phi;      // F: potential address of config 0, -1 logical
    const int64_t *lp_off;       // F+1
    int32_t *flag;               // non-finite read-out flag
    int32_t V, E, F, zero_addr;
    // 0: message rows of two states are packed (one value, m1 - m0, see the
    // kernels); 1: every row holds its states one per panel row (the reverse
    // sweep's adjoint sums, summed by the variable phase like messages)
    int32_t raw_msgs;
};

// A unit of a launch: tile t of graph g (index into the launch's graph array).
struct WorkItem {
    int32_t g;
    int32_t t;
};

}  // namespace lbp
