// First-fit allocator of the server's output arena (host-side bookkeeping
// only: offsets into a device buffer the server owns or was given).  Plain
// C++ with no HIP dependency, so that it can be built and checked on the host
// alone.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace orng {

// First-fit allocator over [0, size) with 256-byte granules.
class Arena {
  public:
    void init(uint64_t size) {
        size_ = size & ~255ull;
        free_.clear();
        if (size_) free_[0] = size_;
        used_ = peak_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = (bytes + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) & ~255ull;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }
    uint64_t peak() const { return peak_; }
    uint64_t used() const { return used_; }

  private:
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

}  // namespace orng
