// First-fit allocator over one block of memory (host bookkeeping only: it
// hands out offsets; the serving engine places its batches' buffers at those
// offsets of one device allocation).  Freed ranges are merged with free
// neighbours, so after every range is released the whole block is one free
// range again.
#pragma once
#include <cstddef>
#include <iterator>
#include <map>

namespace fdfbi {

class Arena {
  public:
    // Forget every allocation; the block is [0, size).
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
    }
    // The lowest free range of at least `bytes` (> 0): its first `bytes` are
    // taken and their offset stored in *off.  False when no free range fits.
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[*off + bytes] = rest;
            return true;
        }
        return false;
    }
    // Return [off, off + bytes), a range alloc handed out.
    void release(size_t off, size_t bytes)
    {
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
    // Free ranges, offset -> length, in offset order.
    const std::map<size_t, size_t> &free_ranges() const { return free_; }

  private:
    std::map<size_t, size_t> free_;
};

}  // namespace fdfbi
