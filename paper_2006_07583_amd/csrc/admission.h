// Admission of served requests (serve.hip): the arena allocator over the
// server's one device allocation and the first-come-first-served rule.
// Host-only C++ (no HIP), so that the policy can be exercised on the CPU
// against a simulated executor.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>

namespace adi {

// First-fit allocator over one device allocation (offsets, 256-byte units).
class Arena {
   public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
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
    size_t used() const { return used_; }
    // free blocks (offset -> size), for checks
    const std::map<size_t, size_t>& free_blocks() const { return free_; }

   private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

// The oldest pending request may start when fewer than max_active requests
// are admitted and its memory fits the arena; the memory is reserved at the
// first check that finds room (off != (size_t)-1 afterwards) and kept while
// the request waits for an admission slot.  No later request overtakes it.
// R has fields `bytes` and `off`.
template <class R>
bool admissible(std::deque<R*>& pending, int64_t admitted, int64_t max_active, Arena& arena) {
    if (pending.empty() || admitted >= max_active) return false;
    R* f = pending.front();
    if (f->off == (size_t)-1) {
        size_t off;
        if (!arena.alloc(f->bytes, &off)) return false;
        f->off = off;
    }
    return true;
}

}  // namespace adi
