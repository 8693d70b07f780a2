// First-fit allocator over an address range [0, size) (internal; used by
// the serving layer for its HBM arena).  Host-only bookkeeping: offsets and
// sizes, no device calls.
#pragma once
#include <stddef.h>

#include <iterator>
#include <map>

namespace hac {

// First-fit allocator over [0, size), coalescing free neighbours.
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
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

    // Free blocks (offset -> bytes), for checks.
    const std::map<size_t, size_t> &free_blocks() const { return free_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> bytes
};

}  // namespace hac
