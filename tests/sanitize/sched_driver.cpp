// CPU driver of the request server's host-side scheduling state (ks_sched.h)
// with a fake executor: built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
//   1. SchedArena against a brute-force model of 256-byte units: first fit
//      (the lowest free offset that fits), no overlap, full coalescing.
//   2. A simulated server: requests with a footprint (resident A plus
//      workspace), a workspace size and a run time in ticks arrive at random
//      ticks; each tick admits first come first served (sched_admits, then
//      SchedPool::place with a malloc-backed fake device allocator), runs,
//      retires the finished requests and releases their workspaces.  Checked
//      every tick: the bytes in use and the segments within the budget, the
//      live workspaces inside their segments and disjoint, free plus live
//      ranges tiling each segment, admission in submission order, and that
//      the head of the queue is held back only by a full slot table, the
//      budget or no place for its workspace (never when nothing is in flight:
//      the segments are then released and the placement retried, so a
//      workspace larger than every segment cannot wait forever); at the end
//      every request has finished, no earlier than its run time after its
//      submission.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <random>
#include <vector>

#include "ks_sched.h"

using namespace ks;

static int failures = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::printf("CHECK failed line %d: %s\n", __LINE__, #c);         \
            if (++failures > 20) std::exit(1);                               \
        }                                                                    \
    } while (0)

static void arena_model_test(uint32_t seed) {
    std::mt19937 rng(seed);
    const size_t units = 64 + rng() % 200;
    SchedArena ar;
    ar.init(units * SCHED_ALIGN);
    std::vector<char> used(units, 0);
    std::map<size_t, size_t> live;  // off -> bytes (aligned)
    for (int op = 0; op < 4000; ++op) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t want = 1 + rng() % (8 * SCHED_ALIGN);
            const size_t u = sched_align(want) / SCHED_ALIGN;
            // model: lowest start with u free units
            long expect = -1;
            for (size_t s = 0; s + u <= units && expect < 0; ++s) {
                bool ok = true;
                for (size_t k = 0; k < u && ok; ++k) ok = !used[s + k];
                if (ok) expect = (long)s;
            }
            size_t off = 0;
            const bool got = ar.alloc(want, &off);
            CHECK(got == (expect >= 0));
            if (got) {
                CHECK(off == (size_t)expect * SCHED_ALIGN);
                for (size_t k = 0; k < u; ++k) {
                    CHECK(!used[off / SCHED_ALIGN + k]);
                    used[off / SCHED_ALIGN + k] = 1;
                }
                live[off] = u * SCHED_ALIGN;
            }
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            ar.release(it->first, it->second);
            for (size_t k = 0; k < it->second / SCHED_ALIGN; ++k) used[it->first / SCHED_ALIGN + k] = 0;
            live.erase(it);
        }
        // the free ranges are exactly the model's maximal free runs
        std::map<size_t, size_t> runs;
        for (size_t s = 0; s < units;) {
            if (used[s]) { ++s; continue; }
            size_t e = s;
            while (e < units && !used[e]) ++e;
            runs[s * SCHED_ALIGN] = (e - s) * SCHED_ALIGN;
            s = e;
        }
        CHECK(runs == ar.free_ranges());
    }
}

struct SimReq {
    int id;
    size_t footprint, ws;
    int run_ticks, submit_tick;
    int start_tick = -1, done_tick = -1, seg = -1;
    size_t off = 0;
};

static void server_sim(uint32_t seed) {
    std::mt19937 rng(seed);
    const size_t budget = (size_t)(2 + rng() % 6) << 30;  // 2..7 GiB
    const int max_inflight = 1 + (int)(rng() % 24);
    SchedPool pool(budget);
    std::vector<void *> fake_device;
    auto dev_alloc = [&](size_t bytes) -> char * {
        // the fake device: host memory of the segment's size is not needed,
        // only a distinct base; a small allocation stands in for it
        void *p = std::malloc(64);
        fake_device.push_back(p);
        return static_cast<char *>(p);
    };
    auto dev_free = [&](char *p) {
        for (auto &q : fake_device)
            if (q == p) {
                std::free(q);
                q = nullptr;
            }
    };
    std::vector<SimReq> reqs;
    const int nreq = 300;
    int t = 0;
    for (int i = 0; i < nreq; ++i) {
        t += (int)(rng() % 3);
        SimReq r{};
        r.id = i;
        // 1..600 MiB, and now and then more than a minimum segment (1 GiB)
        r.ws = rng() % 8 ? (size_t)(1 + rng() % 600) << 20 : (size_t)(1024 + rng() % 1024) << 20;
        r.footprint = r.ws + ((size_t)(rng() % 2048) << 20);       // + resident A
        if (r.footprint > budget) r.footprint = budget;            // oversize: rejected at submit in the server
        if (r.ws > r.footprint) r.ws = r.footprint;
        r.run_ticks = 1 + (int)(rng() % 12);
        r.submit_tick = t;
        reqs.push_back(r);
    }
    std::deque<int> queue;
    std::vector<int> inflight;
    size_t in_use = 0;
    int next_sub = 0, admitted = 0, finished = 0, last_admitted = -1;
    for (int tick = 0; finished < nreq && tick < 100000; ++tick) {
        while (next_sub < nreq && reqs[next_sub].submit_tick <= tick) queue.push_back(next_sub++);
        // admission, first come first served
        while (!queue.empty()) {
            SimReq &r = reqs[queue.front()];
            if (!sched_admits(in_use, r.footprint, budget, (int)inflight.size(), max_inflight)) {
                CHECK((int)inflight.size() >= max_inflight || in_use + r.footprint > budget);
                break;
            }
            if (!pool.place_or_reset(r.ws, inflight.empty(), dev_alloc, dev_free, &r.seg, &r.off)) {
                CHECK(!inflight.empty());  // an idle server always places the head
                break;
            }
            CHECK(r.id == last_admitted + 1);  // nothing overtakes the head
            last_admitted = r.id;
            in_use += r.footprint;
            r.start_tick = tick;
            inflight.push_back(r.id);
            queue.pop_front();
            ++admitted;
        }
        CHECK(in_use <= budget);
        CHECK(pool.total() <= budget);
        // live workspaces inside their segments and disjoint; free + live tile each segment
        const auto &segs = pool.segments();
        for (size_t s = 0; s < segs.size(); ++s) {
            std::map<size_t, size_t> ranges = segs[s].arena.free_ranges();
            for (int id : inflight) {
                const SimReq &r = reqs[id];
                if (r.seg != (int)s) continue;
                CHECK(r.off % SCHED_ALIGN == 0 && r.off + sched_align(r.ws) <= segs[s].bytes);
                CHECK(ranges.emplace(r.off, sched_align(r.ws)).second);
            }
            size_t pos = 0;
            for (const auto &kv : ranges) {
                CHECK(kv.first == pos);
                pos = kv.first + kv.second;
            }
            CHECK(pos == segs[s].bytes);
        }
        // the executor runs every admitted request one tick; the finished retire
        std::vector<int> keep;
        for (int id : inflight) {
            SimReq &r = reqs[id];
            if (tick - r.start_tick + 1 >= r.run_ticks) {
                r.done_tick = tick;
                pool.release(r.seg, r.off, r.ws);
                in_use -= r.footprint;
                ++finished;
            } else {
                keep.push_back(id);
            }
        }
        inflight.swap(keep);
    }
    CHECK(finished == nreq);
    for (const SimReq &r : reqs) CHECK(r.done_tick - r.submit_tick + 1 >= r.run_ticks);
    // every workspace released: each segment is one free range again
    for (const auto &sg : pool.segments()) {
        CHECK(sg.arena.free_ranges().size() == 1);
        CHECK(sg.arena.free_ranges().begin()->second == sg.bytes);
    }
    for (void *p : fake_device) std::free(p);
}

int main() {
    for (uint32_t s = 1; s <= 20; ++s) arena_model_test(s);
    for (uint32_t s = 1; s <= 30; ++s) server_sim(s);
    if (failures) {
        std::printf("%d checks failed\n", failures);
        return 1;
    }
    std::printf("scheduler checks passed\n");
    return 0;
}
