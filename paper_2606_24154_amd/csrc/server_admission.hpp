// server_admission.hpp -- the evaluation server's staging arena and
// admission policy (host code only, no HIP calls).
//
// Arena: offsets into one device allocation, handed out in 256-byte granules
// (the arena's size is rounded down to a whole granule, so every offset is
// 256-byte aligned); first fit from the bottom, or the top end of the
// highest free block that fits (alloc_top); freed neighbours coalesce.
//
// Admission (admit): queued requests enter in arrival order while they fit.
// The first one that does not fit is the blocked head of the line; behind
// it, requests of at most 1/kBackfillFrac of the arena that fit are
// admitted past it (backfill) at the arena's top end, so that the space
// freed below stays in one piece for the head, and at most kMaxBypass of
// them per blocked head: the head then waits only for the requests already
// admitted to finish.  Optionally (max_large > 0) at most max_large "large"
// requests (the caller's flag) are active at once: a large request beyond
// the cap blocks the head of the line like one that does not fit, and a
// small one behind the head is passed over while the cap is reached.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>

namespace nebem {

constexpr int kBackfillFrac = 64;  // requests of at most size / 64 may pass a blocked head
constexpr int kMaxBypass = 64;     // ... and at most this many per blocked head

inline size_t arena_bytes(size_t bytes) { return (bytes + 255) & ~size_t(255); }

struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t s)
    {
        size = s & ~size_t(255);
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = arena_bytes(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return true;
            }
        return false;
    }
    bool alloc_top(size_t bytes, size_t &off)
    {
        bytes = arena_bytes(bytes);
        for (auto it = free_.rbegin(); it != free_.rend(); ++it)
            if (it->second >= bytes) {
                const size_t start = it->first, rest = it->second - bytes;
                off = start + rest;
                free_.erase(std::next(it).base());
                if (rest) free_[start] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = arena_bytes(bytes);
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
};

struct AdmitState {
    int64_t blocked_id = 0;  // id of the blocked head of the line (0: none)
    int bypassed = 0;        // requests admitted past it
    int64_t backfilled = 0;  // requests admitted past any blocked head, in total
    int active_large = 0;    // large requests admitted and not yet finished
};

// R: a request with members id (> 0), bytes, off and large.  Admitted
// requests leave the queue with off set and are passed to on_admit in
// admission order; the caller decrements st.active_large when a large one
// finishes.  max_large <= 0: no cap.  Returns whether any was admitted.
template <class R, class OnAdmit>
bool admit(std::deque<R *> &queue, Arena &arena, AdmitState &st, int max_large, OnAdmit &&on_admit)
{
    bool any = false;
    const R *head = nullptr;
    for (auto it = queue.begin(); it != queue.end();) {
        R *r = *it;
        size_t off;
        const bool capped = r->large && max_large > 0 && st.active_large >= max_large;
        if (!head) {
            if (capped || !arena.alloc(r->bytes, off)) {
                head = r;
                if (st.blocked_id != r->id) {
                    st.blocked_id = r->id;
                    st.bypassed = 0;
                }
                ++it;
                continue;
            }
        } else {
            if (st.bypassed >= kMaxBypass) break;
            if (capped || r->bytes > arena.size / kBackfillFrac || !arena.alloc_top(r->bytes, off)) {
                ++it;
                continue;
            }
            ++st.bypassed;
            ++st.backfilled;
        }
        r->off = off;
        if (r->large) ++st.active_large;
        it = queue.erase(it);
        on_admit(r);
        any = true;
    }
    if (!head) st.blocked_id = 0;
    return any;
}

}  // namespace nebem
