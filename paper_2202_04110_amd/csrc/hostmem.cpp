// Pooled page-locked host memory for graph panels (see hostmem.h).
#include "hostmem.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

namespace lbp {
namespace {

constexpr size_t kHeader = 64;  // keeps the caller's pointer 64-byte aligned
constexpr size_t kMinPinned = size_t(1) << 20;
constexpr uint32_t kPinned = 0x50494e44u, kPlain = 0x504c4e44u;

struct Header {
    uint32_t kind;
    uint32_t pad;
    size_t size_class;
};

struct Pool {
    std::mutex mu;
    std::map<size_t, std::vector<void *>> free_lists;
    size_t pinned = 0;
    bool disabled = false;
};

// Never destroyed: pinned buffers stay valid until the process ends, and no
// HIP call runs during static destruction.
Pool &pool() {
    static Pool *p = new Pool;
    return *p;
}

void *plain(size_t need) {
    void *p = nullptr;
    if (posix_memalign(&p, kHeader, need) != 0) return nullptr;
    Header *h = (Header *)p;
    h->kind = kPlain;
    h->size_class = 0;
    return (char *)p + kHeader;
}

}  // namespace

void *panel_alloc(size_t bytes) {
    const size_t need = bytes + kHeader;
    if (need < kMinPinned) return plain(need);
    size_t c = kMinPinned;
    while (c < need) c <<= 1;
    Pool &P = pool();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto &v = P.free_lists[c];
        if (!v.empty()) {
            void *p = v.back();
            v.pop_back();
            return (char *)p + kHeader;
        }
        if (P.disabled || P.pinned + c > kPinnedPanelCap) return plain(need);
        P.pinned += c;  // reserved before the (slow) allocation
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess || !p) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(P.mu);
        P.pinned -= c;
        P.disabled = true;  // no device or no pinnable memory: plain memory from now on
        return plain(need);
    }
    Header *h = (Header *)p;
    h->kind = kPinned;
    h->size_class = c;
    return (char *)p + kHeader;
}

void panel_free(void *q) {
    if (!q) return;
    void *p = (char *)q - kHeader;
    const Header *h = (const Header *)p;
    if (h->kind == kPinned) {
        Pool &P = pool();
        std::lock_guard<std::mutex> lk(P.mu);
        P.free_lists[h->size_class].push_back(p);
    } else {
        std::free(p);
    }
}

}  // namespace lbp
