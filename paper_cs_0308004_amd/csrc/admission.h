// Host-only pieces of the serving engine that need no device: the best-fit
// arena allocator and the admission rule.  Kept free of HIP so that they can
// be built and tested on their own.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>
#include <set>
#include <utility>
#include <vector>

namespace dpg {

// Best-fit allocator over [0, size) with coalescing; block lengths are
// rounded up to `align`.  A request takes the smallest free block that holds
// it (the lowest such block among equals), found in O(log n) through an index
// of the free blocks by length: a serving arena holds thousands of small
// blocks, and a first-fit walk over the holes in address order cost the
// scheduler most of its time under load.
class Arena {
   public:
    Arena(size_t size, size_t align) : size_(size), align_(align) {
        if (size_ > 0) add_free(0, size_);
    }
    size_t rounded(size_t bytes) const { return (std::max<size_t>(bytes, 1) + align_ - 1) / align_ * align_; }
    // returns false when no free block fits
    bool alloc(size_t bytes, size_t *off) {
        const size_t need = rounded(bytes);
        auto it = by_len_.lower_bound({need, 0});
        if (it == by_len_.end()) return false;
        const size_t at = it->second, len = it->first;
        by_len_.erase(it);
        free_.erase(at);
        if (len > need) add_free(at + need, len - need);
        *off = at;
        used_[at] = need;
        in_use_ += need;
        high_water_ = std::max(high_water_, in_use_);
        return true;
    }
    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t start = off, len = u->second;
        in_use_ -= len;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            by_len_.erase({next->second, next->first});
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                by_len_.erase({prev->second, prev->first});
                free_.erase(prev);
            }
        }
        add_free(start, len);
        return true;
    }
    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t high_water() const { return high_water_; }
    size_t largest_free() const { return by_len_.empty() ? 0 : by_len_.rbegin()->first; }
    size_t free_blocks() const { return free_.size(); }

   private:
    void add_free(size_t at, size_t len) {
        free_[at] = len;
        by_len_.insert({len, at});
    }
    size_t size_, align_;
    size_t in_use_ = 0, high_water_ = 0;
    std::map<size_t, size_t> free_;                // offset -> length
    std::set<std::pair<size_t, size_t>> by_len_;   // (length, offset) of every free block
    std::map<size_t, size_t> used_;                // offset -> length
};

// What admission does with the request at the head of the queue.
enum AdmitKind { ADMIT_OK = 0, ADMIT_WAIT = 1, ADMIT_FAIL = 2 };

struct AdmitResult {
    AdmitKind kind = ADMIT_WAIT;
    size_t out_off = 0, ws_off = 0;
    bool has_out = false, has_ws = false;
};

// Arena bytes a request takes: its output and workspace blocks, each rounded.
inline size_t admit_need(const Arena &a, size_t out_bytes, size_t ws_bytes) {
    return (out_bytes ? a.rounded(out_bytes) : 0) + (ws_bytes ? a.rounded(ws_bytes) : 0);
}

// Admit the head request: reserve its output and workspace.  `capacity` is
// what the arena can ever hold for requests (its size less the blocks the
// server keeps for itself); a request needing more fails at once.  When both
// blocks cannot be reserved now, the request waits -- unless nothing that
// would free memory is pending (`nothing_will_free`: the server is stopping
// with no work in flight), in which case it fails too.  Either failure
// leaves the arena as it was.
inline AdmitResult admit_head(Arena &a, size_t capacity, size_t out_bytes, size_t ws_bytes,
                              bool nothing_will_free) {
    AdmitResult r;
    if (admit_need(a, out_bytes, ws_bytes) > capacity) {
        r.kind = ADMIT_FAIL;
        return r;
    }
    if (out_bytes > 0) {
        if (!a.alloc(out_bytes, &r.out_off)) {
            r.kind = nothing_will_free ? ADMIT_FAIL : ADMIT_WAIT;
            return r;
        }
        r.has_out = true;
    }
    if (ws_bytes > 0) {
        if (!a.alloc(ws_bytes, &r.ws_off)) {
            if (r.has_out) a.release(r.out_off);
            r.has_out = false;
            r.kind = nothing_will_free ? ADMIT_FAIL : ADMIT_WAIT;
            return r;
        }
        r.has_ws = true;
    }
    r.kind = ADMIT_OK;
    return r;
}

// What a free stream slot launches from the admitted queue (flags: for each
// admitted request in admission order, whether a persistent batch can carry
// it).  An unbatched request at the head runs alone; otherwise the batched
// requests of the queue, in order, up to max_batch, form one batch --
// unbatched requests between them keep their place.  Returns the queue
// positions taken (empty for an empty queue).
inline std::vector<size_t> select_launch(const std::vector<bool> &batched, int max_batch) {
    std::vector<size_t> take;
    if (batched.empty()) return take;
    if (!batched[0] || max_batch <= 1) {
        take.push_back(0);
        return take;
    }
    for (size_t i = 0; i < batched.size() && (int)take.size() < max_batch; ++i)
        if (batched[i]) take.push_back(i);
    return take;
}

}  // namespace dpg
