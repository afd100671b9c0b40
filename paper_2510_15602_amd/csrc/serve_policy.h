// Admission policy of the serving loop: a first-fit arena over the server's
// device-memory budget and the rule that forms the next batch from the
// pending requests.  Host-only C++ with no device calls, so that the policy
// can be exercised without a GPU.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace qfca {
namespace serve {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over offsets [0, size); freed ranges are coalesced with
// their neighbours, so a drained arena is again one free range.
class Arena {
public:
    void reset(size_t size) {
        free_.clear();
        size_ = size;
        used_ = peak_ = 0;
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        if (bytes == 0 || bytes > size_) return false;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t o = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[o + bytes] = rest;
            *off = o;
            used_ += bytes;
            if (used_ > peak_) peak_ = used_;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
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
        used_ -= bytes;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t free_ranges() const { return free_.size(); }

private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

// Device working memory of one request of H*W pixels and C channels: bins
// (C bytes per pixel) and the fixed-point channel sum (8 bytes per pixel),
// each 256-byte aligned.
inline size_t request_bytes(int C, int H, int W) {
    const size_t N = (size_t)H * W;
    return align_up((size_t)C * N) + align_up(8 * N);
}

// Moves requests from the front of `pending` into `out` (one batch):
//  * only requests of the head's group (requests that can share a launch);
//    requests of other groups keep their place for a later batch,
//  * in arrival order, while the batch holds fewer than max_batch requests,
//  * each one only if its memory fits in the arena; the first request of
//    the group that does not fit ends the batch, so a large request is never
//    overtaken by later requests of its group (no starvation).
// R needs the members `uint64_t ticket`, `int group`, `size_t bytes` and
// `size_t off`; `off` receives the arena offset.  Returns the number taken;
// *blocked receives the ticket of the request whose memory did not fit, or 0.
template <class R>
size_t form_batch(std::deque<R>& pending, Arena& arena, int max_batch, std::vector<R>& out,
                  uint64_t* blocked) {
    out.clear();
    if (blocked) *blocked = 0;
    if (pending.empty() || max_batch < 1) return 0;
    const int group = pending.front().group;
    for (auto it = pending.begin(); it != pending.end() && (int)out.size() < max_batch;) {
        if (it->group != group) {
            ++it;
            continue;
        }
        size_t off = 0;
        if (!arena.alloc(it->bytes, &off)) {
            if (blocked) *blocked = it->ticket;
            break;
        }
        it->off = off;
        out.push_back(*it);
        it = pending.erase(it);
    }
    return out.size();
}

}  // namespace serve
}  // namespace qfca
