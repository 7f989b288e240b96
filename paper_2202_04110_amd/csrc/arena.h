// First-fit sub-allocator over one contiguous region (host-side bookkeeping
// only; the region itself may be device memory).  Offsets and sizes are
// rounded to 256 bytes; freed blocks coalesce with their neighbours.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <map>

namespace lbp {

class Arena {
public:
    static constexpr size_t kNone = SIZE_MAX;

    explicit Arena(size_t capacity = 0) : cap_(capacity & ~size_t(255)) {
        if (cap_) free_[0] = cap_;
    }

    static size_t round(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) & ~size_t(255); }

    // Offset of a block of at least `bytes`, or kNone.
    size_t alloc(size_t bytes) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return kNone;
    }

    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
    size_t free_blocks() const { return free_.size(); }

private:
    size_t cap_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> size
};

}  // namespace lbp
