// mc_pool.hpp -- first-fit sub-allocator over one device memory pool.
//
// The serving runtime takes its whole device budget once and carves each
// admitted query's memory out of it, so admission is a host-side decision
// (does a block of this size fit now?) and retiring a query returns its block
// without any device allocation call.  Free blocks are kept sorted by offset
// and coalesced with their neighbours on release.  Pure host C++: no device
// calls, offsets only.
#pragma once
#include <cstdint>
#include <iterator>
#include <map>

namespace mc {

class Pool {
   public:
    static constexpr int64_t kAlign = 256;

    explicit Pool(int64_t bytes = 0) { reset(bytes); }

    void reset(int64_t bytes) {
        size_ = bytes > 0 ? bytes - bytes % kAlign : 0;
        free_.clear();
        used_.clear();
        if (size_ > 0) free_[0] = size_;
        in_use_ = 0;
        peak_ = 0;
    }

    static int64_t round_up(int64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

    // First-fit allocation; returns the offset or -1 when no free block is large enough.
    int64_t alloc(int64_t bytes) {
        if (bytes <= 0) bytes = kAlign;
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_[off] = bytes;
            in_use_ += bytes;
            if (in_use_ > peak_) peak_ = in_use_;
            return off;
        }
        return -1;
    }

    // Release a block returned by alloc; false if the offset is not a live block.
    bool release(int64_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        int64_t start = off, len = u->second;
        in_use_ -= len;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
        return true;
    }

    int64_t size() const { return size_; }
    int64_t in_use() const { return in_use_; }
    int64_t peak() const { return peak_; }
    int64_t largest_free() const {
        int64_t m = 0;
        for (auto &f : free_) m = f.second > m ? f.second : m;
        return m;
    }
    size_t n_free_blocks() const { return free_.size(); }
    size_t n_used_blocks() const { return used_.size(); }

   private:
    int64_t size_ = 0, in_use_ = 0, peak_ = 0;
    std::map<int64_t, int64_t> free_;  // offset -> length
    std::map<int64_t, int64_t> used_;  // offset -> length
};

}  // namespace mc
