// First-fit allocator over one contiguous device range [0, size): host-side
// bookkeeping only (offsets, no pointers), so it builds and is tested
// without a GPU.  Blocks are aligned to `align` bytes; freed blocks are
// coalesced with their free neighbours.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <map>

namespace pyro {

class Arena {
public:
    static constexpr size_t kNone = SIZE_MAX;

    explicit Arena(size_t size = 0, size_t align = 256) : size_(size / align * align), align_(align)
    {
        if (size_ > 0) free_[0] = size_;
    }

    // Offset of a new block of at least `bytes` bytes, or kNone.
    size_t alloc(size_t bytes)
    {
        if (bytes == 0) bytes = 1;
        const size_t need = (bytes + align_ - 1) / align_ * align_;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            live_[off] = need;
            used_ += need;
            return off;
        }
        return kNone;
    }

    // Release the block at `off`; false if no live block starts there.
    bool release(size_t off)
    {
        auto it = live_.find(off);
        if (it == live_.end()) return false;
        size_t start = off, len = it->second;
        live_.erase(it);
        used_ -= len;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
        return true;
    }

    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t live_blocks() const { return live_.size(); }
    size_t free_blocks() const { return free_.size(); }
    size_t largest_free() const
    {
        size_t m = 0;
        for (auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

private:
    size_t size_, align_, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> live_;  // offset -> length
};

}  // namespace pyro
