// Host-side range allocator of the serving pool (vertex, entry and tile
// ranges).  Plain C++, no HIP: also compiled on its own by the test suite.
#pragma once

#include <climits>
#include <cstdint>
#include <iterator>
#include <map>
#include <utility>

namespace fsv {

// First-fit allocator over [0, cap) with coalescing of freed ranges.  First
// fit keeps the live ranges low in the pool, which bounds the vertex range the
// per-step pool-wide kernels cover.
class RangeAlloc {
public:
    explicit RangeAlloc(int64_t cap = 0) { reset(cap); }
    void reset(int64_t cap) {
        free_.clear();
        cap_ = cap;
        if (cap > 0) free_[0] = cap;
    }
    int64_t alloc(int64_t len) {
        if (len <= 0) return 0;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                const int64_t start = it->first, rest = it->second - len;
                free_.erase(it);
                if (rest > 0) free_[start + len] = rest;
                return start;
            }
        }
        return -1;
    }
    void release(int64_t start, int64_t len) {
        if (len <= 0) return;
        auto it = free_.emplace(start, len).first;
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
    int64_t capacity() const { return cap_; }

private:
    std::map<int64_t, int64_t> free_;  // start -> length
    int64_t cap_ = 0;
};

}  // namespace fsv
