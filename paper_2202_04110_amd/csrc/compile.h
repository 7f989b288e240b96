// Host-side validation of an lbp_graph_desc and its compilation into the
// 64-lane panel layout described in lbp_internal.h.
#pragma once

#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lbp.h"
#include "hostmem.h"
#include "lbp_internal.h"

namespace lbp {

// Factor tiles launched together: same kernel, same shape.  TK_LOGL groups
// hold every logical tile of at most 256 edges (lane- and wavefront-per-factor
// tiles share one kernel); TK_LOGW groups hold the wider ones.
struct FGroup {
    int32_t kind;  // TK_*
    int32_t a, b;  // PAIR: slot state counts; otherwise 0
    std::vector<int32_t> tiles;
};

// Variable tiles launched together in the low-degree belief kernel.
struct VGroup {
    int32_t bucket;  // register bucket: max states over the tiles' low-degree lanes
    std::vector<int32_t> tiles;
};

// Allocator of the host panels: storage from panel_alloc (page-locked when
// possible) and default-initialised elements, so resize() leaves them
// unwritten (panels are filled completely afterwards).
template <class T>
struct PanelAllocator {
    using value_type = T;
    PanelAllocator() = default;
    template <class U>
    PanelAllocator(const PanelAllocator<U> &) noexcept {}
    T *allocate(size_t n) {
        void *p = panel_alloc(n * sizeof(T));
        if (!p) throw std::bad_alloc();
        return (T *)p;
    }
    void deallocate(T *p, size_t) noexcept { panel_free(p); }
    template <class U>
    void construct(U *p) noexcept {
        ::new ((void *)p) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
    template <class U>
    bool operator==(const PanelAllocator<U> &) const noexcept {
        return true;
    }
    template <class U>
    bool operator!=(const PanelAllocator<U> &) const noexcept {
        return false;
    }
};
using PanelBuf = std::vector<float, PanelAllocator<float>>;

struct HostLayout {
    int64_t V = 0, VS = 0, F = 0, E = 0, ES = 0, Tn = 0;
    int64_t M = 0, VB = 0, P = 0;  // floats in the message, belief and potential arrays
    int32_t zero_addr = 0;
    std::vector<FTile> ftile;
    std::vector<int32_t> fvb;
    std::vector<int32_t> fvar;  // variable of each (tile, slot, lane), same indexing as fvb (-1 idle)
    std::vector<int32_t> faff;  // [tile][2]: first variable of a lane-contiguous pairwise slot, else -1
    bool fusable = false;       // every variable on the lane path, every factor dense pairwise
    std::vector<VTile> vtile;
    std::vector<int32_t> vedge, vns;
    std::vector<HVar> hvar;
    std::vector<int32_t> hedge;
    std::vector<int32_t> mids, highs;  // indices into hvar: wavefront- / block-per-variable paths
    std::vector<int32_t> cols;         // indices into hvar: column groups (block path)
    std::vector<GenClass> gcls;
    std::vector<uint8_t> grows;
    std::vector<int32_t> edge_maddr;
    // Variables are laid out in an internal order (see compile_desc): vn,
    // vs_off and every tile array are indexed by internal id, vs_off holds
    // each variable's offset in the caller's flat order, and vext maps an
    // internal id to the caller's (empty when the two orders agree).
    std::vector<int64_t> es_off, vs_off;
    std::vector<int32_t> vn, fac_phi, vext;
    std::vector<int64_t> lp_off;
    PanelBuf theta_panel, phi_panel;  // every element written by compile_desc (or fill_panels)
    std::vector<int32_t> tile_fac;    // factor of each (tile, lane) with a potential panel, -1 otherwise
                                      // (kept only when compile_desc leaves the panels to fill_panels)
    std::vector<FGroup> fgroups;
    std::vector<VGroup> vgroups;
};

// Returns LBP_OK or an LBP_E_* code with a message in *err.
// scan_potentials = false leaves the NaN/infinity check of the log-potentials
// to the caller (compile_desc does it while filling the potential panels).
int validate_desc(const lbp_graph_desc *d, int64_t sizes[6], std::string *err, bool scan_potentials = true);
// fill = false: the layout without its evidence and potential panels, which
// fill_panels then writes wherever the caller wants them (an upload image).
int compile_desc(const lbp_graph_desc *d, HostLayout *L, std::string *err, bool fill = true);
// Writes the evidence panel (L.VB floats) and the potential panel (L.P
// floats) of a layout compiled from `d`, checking the potentials for NaN and
// infinity (LBP_E_INVALID naming the first).
int fill_panels(const lbp_graph_desc *d, const HostLayout &L, float *theta, float *phi, std::string *err);
// LBP_E_INVALID naming the first NaN or infinite log-potential of `d`, else
// LBP_OK (the check fill_panels makes on its way, for callers that leave the
// panels to the device).
int check_potentials_finite(const lbp_graph_desc *d, int64_t Tn, std::string *err);
// Copies n floats and returns the index of the first NaN or infinity among
// them, or -1 (one pass over the source).
int64_t copy_check_finite(float *dst, const float *src, int64_t n);
// LBP_E_INVALID naming log_potentials[i] as not finite.
int nonfinite_potential(int64_t i, std::string *err);
// Host replay of every kernel's addresses against the layout's array sizes.
int check_layout(const HostLayout &L, std::string *err);

// Bucket of the low-degree belief kernel for a tile whose low lanes have at
// most n states.
inline int32_t state_bucket(int32_t n) { return n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : 16; }
// Chunk bucket of the wave-per-factor logical kernel.
inline int32_t chunk_bucket(int32_t chunks) { return chunks <= 1 ? 1 : chunks <= 4 ? 4 : 16; }

}  // namespace lbp
