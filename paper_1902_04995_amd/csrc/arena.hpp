// First-fit sub-allocator over a fixed byte range, with coalescing of
// neighbouring free blocks.  Host-side bookkeeping only (it never touches the
// memory it manages), so the serving loop can carve one device buffer into
// per-micro-batch blocks without calling the device allocator.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace rgb {

class Arena {
public:
    explicit Arena(uint64_t capacity = 0, uint64_t align = 256) : cap_(capacity), align_(align ? align : 1) {
        if (cap_) free_[0] = cap_;
    }

    uint64_t capacity() const { return cap_; }
    uint64_t in_use() const { return used_; }

    uint64_t rounded(uint64_t n) const { return (n + align_ - 1) / align_ * align_; }

    // Largest block that could be handed out right now.
    uint64_t largest_free() const {
        uint64_t best = 0;
        for (const auto& kv : free_)
            if (kv.second > best) best = kv.second;
        return best;
    }

    // Offset of a block of at least n bytes, or UINT64_MAX if none fits.
    uint64_t alloc(uint64_t n) {
        n = rounded(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            uint64_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[off + n] = sz - n;
            used_blocks_[off] = n;
            used_ += n;
            return off;
        }
        return UINT64_MAX;
    }

    // Return a block; false if `off` is not the start of a live block.
    bool release(uint64_t off) {
        auto u = used_blocks_.find(off);
        if (u == used_blocks_.end()) return false;
        uint64_t sz = u->second;
        used_blocks_.erase(u);
        used_ -= sz;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + sz == next->first) {
            sz += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += sz;
                return true;
            }
        }
        free_[off] = sz;
        return true;
    }

    // Invariant check (tests): free and used blocks tile [0, capacity) exactly,
    // and no two free blocks touch.
    bool consistent() const {
        std::map<uint64_t, std::pair<uint64_t, bool>> all;
        for (const auto& kv : free_) all[kv.first] = {kv.second, true};
        for (const auto& kv : used_blocks_) {
            if (all.count(kv.first)) return false;
            all[kv.first] = {kv.second, false};
        }
        uint64_t pos = 0, used = 0;
        bool prev_free = false;
        for (const auto& kv : all) {
            if (kv.first != pos || kv.second.first == 0) return false;
            if (kv.second.second && prev_free) return false;
            prev_free = kv.second.second;
            if (!kv.second.second) used += kv.second.first;
            pos += kv.second.first;
        }
        return pos == cap_ && used == used_;
    }

private:
    uint64_t cap_ = 0, align_ = 1, used_ = 0;
    std::map<uint64_t, uint64_t> free_;         // offset -> size
    std::map<uint64_t, uint64_t> used_blocks_;  // offset -> size
};

}  // namespace rgb
