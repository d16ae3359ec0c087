// Scheduler of the serving loop: arrivals, HBM-arena admission, continuous
// batching over a fixed number of stream slots, completions, time-outs.
// Independent of HIP: an executor supplies the clock, the launch, the
// completion query and the idle wait, so the same loop drives the GPU and a
// simulated device (for CPU tests and capacity planning).
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

#include "../../include/utf16wf.h"
#include "../../include/utf16wf_serve.h"

namespace utf16wf {
namespace serve {

constexpr int32_t kStatusPending = 2;
constexpr int32_t kStatusTimedOut = 1;

// First-fit allocator over [0, total) with coalescing frees; 256-byte
// granularity.
class Arena {
  public:
    explicit Arena(int64_t total) : total_(total) {
        if (total > 0)
            free_[0] = total;
    }
    static int64_t round_up(int64_t b) { return (b + 255) & ~int64_t(255); }

    int64_t alloc(int64_t bytes) {
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0)
                    free_[off + bytes] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return off;
            }
        }
        return -1;
    }

    void release(int64_t off, int64_t bytes) {
        bytes = round_up(bytes);
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

    int64_t largest_free() const {
        int64_t m = 0;
        for (const auto &kv : free_)
            m = std::max(m, kv.second);
        return m;
    }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
    int64_t total() const { return total_; }

  private:
    std::map<int64_t, int64_t> free_;
    int64_t total_ = 0, used_ = 0, peak_ = 0;
};

// Layout of one batch inside its arena region: packed input units, output
// units, uint8 results[B], each 256-byte aligned. The output part has 16
// bytes per request to spare, so that a request's output can start at its
// input's address phase. (The batch's offsets and copy descriptors travel in
// a small per-slot staging buffer.)
struct BatchLayout {
    int64_t in_off, out_off, results_off, bytes;
};

inline BatchLayout layout(int64_t nreq, int64_t units) {
    BatchLayout l;
    l.in_off = 0;
    l.out_off = Arena::round_up(units * 2);
    l.results_off = l.out_off + Arena::round_up(units * 2 + 16 * nreq);
    l.bytes = l.results_off + Arena::round_up(nreq > 0 ? nreq : 1);
    return l;
}

struct Batch {
    int64_t id = -1;
    int slot = -1;
    std::vector<int64_t> reqs;
    int64_t units = 0;
    int64_t region = -1;
    BatchLayout lay{};
};

struct Request {
    int64_t arrival_ns;
    int64_t length;
};

// Executor interface (duck-typed):
//   int64_t now();
//   int launch(Batch &b);             // 0 or a negative status
//   int done(int slot);               // 1 when the slot's batch finished, 0 not yet, <0 failed
//   void finish(const Batch &b, utf16wf_serve_outcome *out);
//   void idle(int64_t next_arrival_ns /* -1 none */, bool any_busy);
//   void drain(int slot);             // after a failed launch: wait for what it
//                                     // queued on the slot before it failed
template <class Exec>
int run_loop(Exec &ex, const utf16wf_serve_config &cfg, const Request *rq, int64_t n,
             utf16wf_serve_outcome *out, utf16wf_serve_stats *st) {
    Arena arena(cfg.arena_bytes);
    std::deque<int64_t> queue;
    const int slots = cfg.num_streams;
    std::vector<Batch> inflight(slots);
    std::vector<bool> busy(slots, false);
    int64_t next = 0, finished = 0, nbusy = 0;
    int64_t batch_id = 0;
    utf16wf_serve_stats s{};
    for (int64_t i = 0; i < n; ++i)
        out[i] = utf16wf_serve_outcome{-1, -1, kStatusPending, -1, -1, cfg.op == UTF16WF_OP_IS ? 0 : -1};

    while (finished < n) {
        bool progress = false;
        int64_t now = ex.now();
        while (next < n && rq[next].arrival_ns <= now) {
            queue.push_back(next++);
            progress = true;
        }
        s.max_queue = std::max<int64_t>(s.max_queue, (int64_t)queue.size());

        for (int sl = 0; sl < slots; ++sl) {
            if (!busy[sl])
                continue;
            const int d = ex.done(sl);
            if (d == 0)
                continue;
            const int64_t t = ex.now();
            Batch &b = inflight[sl];
            if (d > 0)
                ex.finish(b, out);
            for (int64_t r : b.reqs) {
                out[r].done_ns = t;
                out[r].status = d > 0 ? 0 : UTF16WF_EHIP;
            }
            if (d > 0)
                s.completed += (int64_t)b.reqs.size();
            else
                s.failed += (int64_t)b.reqs.size();
            s.wall_ns = std::max(s.wall_ns, t);
            finished += (int64_t)b.reqs.size();
            arena.release(b.region, b.lay.bytes);
            busy[sl] = false;
            --nbusy;
            progress = true;
        }

        if (cfg.timeout_ns > 0) {
            while (!queue.empty() && now - rq[queue.front()].arrival_ns > cfg.timeout_ns) {
                out[queue.front()].status = kStatusTimedOut;
                queue.pop_front();
                ++s.timed_out;
                ++finished;
                progress = true;
            }
        }

        for (int sl = 0; sl < slots && !queue.empty(); ++sl) {
            if (busy[sl])
                continue;
            Batch b;
            b.slot = sl;
            while (!queue.empty() && (int64_t)b.reqs.size() < cfg.max_batch_requests) {
                const int64_t r = queue.front();
                const int64_t len = rq[r].length;
                if (layout(1, len).bytes > arena.total()) {
                    out[r].status = UTF16WF_ERANGE;  // can never fit
                    queue.pop_front();
                    ++s.rejected;
                    ++finished;
                    progress = true;
                    continue;
                }
                if (!b.reqs.empty() && b.units + len > cfg.max_batch_units)
                    break;
                if (layout((int64_t)b.reqs.size() + 1, b.units + len).bytes > arena.largest_free())
                    break;  // wait until memory frees up; keep arrival order
                b.reqs.push_back(r);
                b.units += len;
                queue.pop_front();
            }
            if (b.reqs.empty())
                break;
            b.lay = layout((int64_t)b.reqs.size(), b.units);
            b.region = arena.alloc(b.lay.bytes);
            b.id = batch_id++;
            const int64_t t = ex.now();
            const int rc = (b.region >= 0) ? ex.launch(b) : UTF16WF_ENOMEM;
            for (int64_t r : b.reqs) {
                out[r].launch_ns = t;
                out[r].batch = (int32_t)(b.id & 0x7FFFFFFF);  // (wraps past 2^31 batches)
                out[r].slot = sl;
            }
            ++s.batches;
            progress = true;
            if (rc != UTF16WF_OK) {
                for (int64_t r : b.reqs) {
                    out[r].status = UTF16WF_EHIP;
                    out[r].done_ns = t;
                }
                s.failed += (int64_t)b.reqs.size();
                finished += (int64_t)b.reqs.size();
                if (b.region >= 0) {
                    // a launch can fail after part of the batch (a copy, the
                    // gather) is queued; that work may still write the region,
                    // so it is freed only once the slot's queue has drained
                    ex.drain(sl);
                    arena.release(b.region, b.lay.bytes);
                }
                continue;
            }
            inflight[sl] = std::move(b);
            busy[sl] = true;
            ++nbusy;
            s.max_inflight = std::max<int64_t>(s.max_inflight, nbusy);
        }
        if (!progress && finished < n)
            ex.idle(next < n ? rq[next].arrival_ns : -1, nbusy > 0);
    }
    s.arena_peak_bytes = arena.peak();
    if (st)
        *st = s;
    return UTF16WF_OK;
}

}  // namespace serve
}  // namespace utf16wf
