// Host buffers for the large per-graph panels built on the host (potentials,
// evidence): page-locked when possible, so their upload runs as a direct DMA
// instead of through the runtime's bounce buffers.
#pragma once

#include <cstddef>

namespace lbp {

// At least `bytes` bytes.  Buffers of 1 MiB and more come from a process-wide
// pool of page-locked host memory (power-of-two size classes, at most
// kPinnedPanelCap bytes pinned in total, kept for reuse until the process
// ends); smaller requests, requests beyond the cap and hosts where page-locked
// allocation fails get ordinary memory.  Returns nullptr only when both fail.
void *panel_alloc(size_t bytes);
// Returns a buffer from panel_alloc (nullptr is ignored).
void panel_free(void *p);

constexpr size_t kPinnedPanelCap = size_t(4) << 30;

}  // namespace lbp
