// Ring of contiguous blocks over positions [0, capacity), handed out and
// given back in FIFO order (a block may be released early; its space is
// reused once every older block is released too).  A block that does not
// fit before the end wraps to position 0; the skipped tail counts as used
// until the block is freed.  Host-side bookkeeping only: the server keeps
// queued requests in pinned host rings with it, so a request is copied once,
// at submission, and consecutive requests sit next to each other.
#pragma once

#include <cstdint>
#include <deque>

namespace rgb {

class Ring {
public:
    explicit Ring(int64_t capacity = 0) : cap_(capacity) {}

    int64_t capacity() const { return cap_; }
    int64_t used() const { return used_; }
    size_t blocks() const { return blocks_.size(); }
    int64_t head() const { return head_; }  // next position handed out (tests)
    int64_t tail() const { return tail_; }  // start of the oldest live block's space (tests)

    // Reserve n contiguous positions; returns the block's id (its index in
    // allocation order) and its first position, or false if it does not fit now.
    bool alloc(int64_t n, int64_t& pos, uint64_t& id) {
        if (n < 0 || n > cap_) return false;
        if (used_ == 0) head_ = tail_ = 0;
        const bool wrapped = used_ > 0 && head_ <= tail_;
        int64_t pad = 0;
        if (!wrapped) {
            if (cap_ - head_ >= n) {
                pos = head_;
            } else if (tail_ >= n) {
                pad = cap_ - head_;
                pos = 0;
            } else {
                return false;
            }
        } else {
            if (tail_ - head_ < n) return false;
            pos = head_;
        }
        head_ = pos + n;
        used_ += n + pad;
        id = next_id_++;
        blocks_.push_back(Block{pos, n, pad, false});
        return true;
    }

    // Give back block `id`; false if it is not live.
    bool release(uint64_t id) {
        if (id < first_id_ || id >= next_id_) return false;
        Block& b = blocks_[(size_t)(id - first_id_)];
        if (b.released) return false;
        b.released = true;
        while (!blocks_.empty() && blocks_.front().released) {
            const Block f = blocks_.front();
            blocks_.pop_front();
            ++first_id_;
            used_ -= f.n + f.pad;
            if (f.n + f.pad > 0) tail_ = f.pos + f.n;  // an empty block holds no space to hand back
        }
        if (used_ == 0) head_ = tail_ = 0;
        return true;
    }

    // Invariant check (tests): live blocks are disjoint, in order around the
    // ring, and their sizes plus pads add up to used().  Empty blocks hold no
    // space and may sit anywhere.
    bool consistent() const {
        int64_t sum = 0;
        for (const Block& b : blocks_) {
            if (b.pos < 0 || b.n < 0 || b.pad < 0 || b.pos + b.n > cap_) return false;
            sum += b.n + b.pad;
        }
        if (sum != used_ || used_ > cap_) return false;
        const Block* p = nullptr;
        for (const Block& c : blocks_) {
            if (c.n == 0) continue;
            if (p) {
                const int64_t end = p->pos + p->n;
                if (c.pad == 0 ? c.pos != end : (c.pos != 0 || end + c.pad != cap_)) return false;
            }
            p = &c;
        }
        return true;
    }

private:
    struct Block {
        int64_t pos, n, pad;
        bool released;
    };
    int64_t cap_ = 0, head_ = 0, tail_ = 0, used_ = 0;
    uint64_t first_id_ = 0, next_id_ = 0;
    std::deque<Block> blocks_;
};

}  // namespace rgb
