// Host-side scheduling state of the request server, free of device calls so
// that it builds and runs on the CPU alone (the server drives it with its
// device allocator; a CPU test drives it with a fake one):
//   SchedArena    first-fit allocator over one segment, in SCHED_ALIGN-byte
//                 units, coalescing neighbouring free ranges;
//   SchedPool     workspaces of admitted requests: first fit in the existing
//                 segments, else a new segment of at least SCHED_SEG_MIN
//                 bytes while all segments together stay within the budget
//                 (and, with nothing in flight, the segments released and
//                 the placement tried again);
//   sched_admits  the first-come-first-served admission rule: the request at
//                 the head of the queue is admitted while the slots and the
//                 budget (resident A plus workspace: its footprint) allow and
//                 a workspace can be placed; nothing overtakes it.
#pragma once
#include <stddef.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <vector>

namespace ks {

constexpr size_t SCHED_ALIGN = 256;
constexpr size_t SCHED_SEG_MIN = (size_t)1 << 30;

inline size_t sched_align(size_t v) { return (v + SCHED_ALIGN - 1) / SCHED_ALIGN * SCHED_ALIGN; }

class SchedArena {
   public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = sched_align(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rem = it->second - bytes, noff = it->first + bytes;
                free_.erase(it);
                if (rem) free_[noff] = rem;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = sched_align(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    // the free ranges (offset -> bytes), for tests
    const std::map<size_t, size_t> &free_ranges() const { return free_; }

   private:
    std::map<size_t, size_t> free_;
};

struct SchedSegment {
    char *base = nullptr;
    size_t bytes = 0;
    SchedArena arena;
};

class SchedPool {
   public:
    explicit SchedPool(size_t budget = 0) : budget_(budget) {}
    void set_budget(size_t budget) { budget_ = budget; }
    // A workspace of `bytes`: first fit in the segments, else a new segment
    // from dev_alloc(size) -> base or nullptr, if the budget allows.  False
    // (nothing allocated) when neither works.
    template <typename DevAlloc>
    bool place(size_t bytes, DevAlloc dev_alloc, int *seg, size_t *off) {
        for (size_t i = 0; i < segs_.size(); ++i) {
            if (segs_[i].arena.alloc(bytes, off)) {
                *seg = (int)i;
                return true;
            }
        }
        const size_t need = sched_align(bytes);
        if (total_ + need > budget_) return false;
        const size_t sz = std::min(std::max(need, SCHED_SEG_MIN), sched_align(budget_ - total_));
        if (sz < need) return false;
        SchedSegment sg;
        sg.base = dev_alloc(sz);
        if (!sg.base) return false;
        sg.bytes = sz;
        sg.arena.init(sz);
        sg.arena.alloc(bytes, off);
        segs_.push_back(sg);
        total_ += sz;
        *seg = (int)segs_.size() - 1;
        return true;
    }
    // place(), and when that fails while no workspace is live (`idle`), all
    // segments returned through dev_free(base) and place() once more: without
    // this a workspace larger than every segment, with the segments already
    // at the budget, would wait forever
    template <typename DevAlloc, typename DevFree>
    bool place_or_reset(size_t bytes, bool idle, DevAlloc dev_alloc, DevFree dev_free, int *seg, size_t *off) {
        if (place(bytes, dev_alloc, seg, off)) return true;
        if (!idle || segs_.empty()) return false;
        for (const SchedSegment &sg : segs_) dev_free(sg.base);
        segs_.clear();
        total_ = 0;
        return place(bytes, dev_alloc, seg, off);
    }
    void release(int seg, size_t off, size_t bytes) { segs_[seg].arena.release(off, bytes); }
    char *base(int seg) const { return segs_[seg].base; }
    const std::vector<SchedSegment> &segments() const { return segs_; }
    size_t total() const { return total_; }

   private:
    size_t budget_ = 0, total_ = 0;
    std::vector<SchedSegment> segs_;
};

// Whether the head of the queue may be admitted before its workspace is
// placed: a free slot and room in the budget for its footprint.
inline bool sched_admits(size_t in_use, size_t footprint, size_t budget, int inflight, int max_inflight) {
    return inflight < max_inflight && in_use + footprint <= budget;
}

}  // namespace ks
