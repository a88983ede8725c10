// Byte-range allocator for one device allocation (host-side bookkeeping only;
// nothing here touches the device).  Blocks are multiples of 256 bytes at
// 256-byte aligned offsets; allocation is best fit, and released ranges merge
// with their free neighbours.
#pragma once
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace gf2x {

class Arena {
   public:
    static constexpr size_t npos = ~(size_t)0;

    explicit Arena(size_t bytes = 0) { reset(bytes); }

    void reset(size_t bytes) {
        free_.clear();
        cap_ = bytes & ~(size_t)255;
        used_ = 0;
        if (cap_) free_[0] = cap_;
    }

    static size_t round(size_t bytes) { return bytes ? (bytes + 255) & ~(size_t)255 : 256; }

    // Offset of a block of round(bytes) bytes, or npos when no free range holds it.
    size_t alloc(size_t bytes) {
        const size_t need = round(bytes);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= need && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return npos;
        const size_t off = best->first, len = best->second;
        free_.erase(best);
        if (len > need) free_[off + need] = len - need;
        used_ += need;
        return off;
    }

    // Returns a block obtained from alloc(bytes) at `off`.
    void release(size_t off, size_t bytes) {
        size_t len = round(bytes);
        used_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return;
            }
        }
        free_[off] = len;
    }

    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t free_ranges() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& f : free_) m = f.second > m ? f.second : m;
        return m;
    }

   private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t cap_ = 0, used_ = 0;
};

}  // namespace gf2x
