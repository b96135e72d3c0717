// First-fit allocator of byte ranges inside one pre-allocated block (host bookkeeping only;
// the block itself, e.g. a device allocation, is owned by the caller).
//
// The serving loop allocates every job's device memory (graph, coordinates, loss history,
// workspace) from one block of the configured budget, so admission never calls the
// device allocator and the budget is a hard bound.  Free ranges are kept ordered by
// offset and merged with their neighbours on release, so a released range is reusable at
// its full size at once.  Plain C++ (no HIP), so it is tested on the host.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace gempe {

class Arena {
public:
    static constexpr size_t kNone = ~size_t(0);

    explicit Arena(size_t capacity = 0, size_t align = 256) { reset(capacity, align); }

    void reset(size_t capacity, size_t align = 256) {
        align_ = align ? align : 1;
        capacity_ = capacity - capacity % align_;
        free_.clear();
        live_.clear();
        used_ = peak_ = 0;
        if (capacity_) free_[0] = capacity_;
    }

    size_t round(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

    // Offset of a range of at least `bytes` (rounded up to the alignment), or kNone.
    size_t alloc(size_t bytes) {
        if (bytes == 0) bytes = 1;
        const size_t need = round(bytes);
        if (need < bytes) return kNone;  // overflow
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, rest = it->second - need;
            free_.erase(it);
            if (rest) free_[off + need] = rest;
            live_[off] = need;
            used_ += need;
            if (used_ > peak_) peak_ = used_;
            return off;
        }
        return kNone;
    }

    // Releases a range returned by alloc; false (and no change) for an unknown offset.
    bool release(size_t off) {
        auto lv = live_.find(off);
        if (lv == live_.end()) return false;
        size_t start = off, size = lv->second;
        used_ -= size;
        live_.erase(lv);
        auto next = free_.lower_bound(start);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.lower_bound(start);
        if (next != free_.end() && start + size == next->first) {
            size += next->second;
            free_.erase(next);
        }
        free_[start] = size;
        return true;
    }

    size_t capacity() const { return capacity_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t live_count() const { return live_.size(); }
    size_t free_ranges() const { return free_.size(); }
    size_t largest_free() const {
        size_t best = 0;
        for (const auto &f : free_)
            if (f.second > best) best = f.second;
        return best;
    }

private:
    size_t align_ = 256, capacity_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> size, disjoint, no two adjacent
    std::map<size_t, size_t> live_;  // offset -> size
};

}  // namespace gempe
