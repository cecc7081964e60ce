// range_alloc.h -- first-fit sub-allocation of byte ranges inside one fixed pool, with
// coalescing of neighbouring free ranges.  Host-side bookkeeping only (the pool itself is
// device or pinned memory owned elsewhere); not thread-safe.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace qc {

class RangeAllocator {
public:
    explicit RangeAllocator(size_t capacity = 0, size_t align = 256) { reset(capacity, align); }

    void reset(size_t capacity, size_t align = 256) {
        align_ = align;
        capacity_ = capacity - capacity % align;
        used_ = 0;
        free_.clear();
        if (capacity_ > 0) free_[0] = capacity_;
    }

    // Bytes rounded up to the alignment.
    size_t rounded(size_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }

    // Takes the first free range that fits; false if none does.
    bool alloc(size_t bytes, size_t* offset) {
        const size_t need = rounded(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *offset = it->first;
            const size_t rest = it->second - need;
            const size_t start = it->first + need;
            free_.erase(it);
            if (rest > 0) free_[start] = rest;
            used_ += need;
            return true;
        }
        return false;
    }

    // Returns a range obtained from alloc() with the same byte count.
    void release(size_t offset, size_t bytes) {
        size_t size = rounded(bytes == 0 ? 1 : bytes);
        used_ -= size;
        auto next = free_.lower_bound(offset);
        if (next != free_.end() && offset + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == offset) {
                prev->second += size;
                return;
            }
        }
        free_[offset] = size;
    }

    size_t capacity() const { return capacity_; }
    size_t used() const { return used_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t free_ranges() const { return free_.size(); }

private:
    std::map<size_t, size_t> free_;   // offset -> size
    size_t capacity_ = 0, used_ = 0, align_ = 256;
};

}  // namespace qc
