// Simulated executor of the serving loop: a virtual clock, a latency model
// per batch and injected launch failures, for testing the scheduler of
// serve_core.h on a CPU and for capacity planning. Free of HIP, so that it
// also builds with a plain host compiler (the sanitizer build of the tests).
#pragma once

#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "serve_core.h"

namespace utf16wf {
namespace serve {

class SimExec {
  public:
    SimExec(int slots, int64_t base, double per_unit, int64_t fail_every)
        : done_at_(slots, 0), base_(base), per_unit_(per_unit), fail_every_(fail_every) {}
    int64_t now() const { return t_; }
    // A simulated failure happens after the batch's work is queued (as a real
    // launch can fail after its copies are on the stream): that work keeps
    // its region busy until it would have completed. Every launch checks that
    // its region does not overlap one that such work may still write.
    int launch(Batch &b) {
        ++launches_;
        for (const Pending &q : pending_)
            if (q.until > t_ && b.region < q.region + q.bytes && q.region < b.region + b.lay.bytes)
                ++hazards_;
        done_at_[b.slot] = t_ + base_ + (int64_t)(per_unit_ * (double)b.units);
        if (fail_every_ > 0 && launches_ % fail_every_ == 0) {
            pending_.push_back(Pending{b.region, b.lay.bytes, done_at_[b.slot]});
            return UTF16WF_EHIP;
        }
        return UTF16WF_OK;
    }
    int done(int slot) { return t_ >= done_at_[slot] ? 1 : 0; }
    void finish(const Batch &, utf16wf_serve_outcome *) {}
    void drain(int slot) { t_ = std::max(t_, done_at_[slot]); }
    void idle(int64_t next_arrival, bool any_busy) {
        int64_t t = INT64_MAX;
        if (next_arrival >= 0)
            t = next_arrival;
        if (any_busy)
            for (int64_t d : done_at_)
                if (d > t_)
                    t = std::min(t, d);
        t_ = (t == INT64_MAX) ? t_ + 1 : std::max(t, t_ + 1);
    }
    int64_t hazards() const { return hazards_; }

  private:
    struct Pending {
        int64_t region, bytes, until;
    };
    std::vector<int64_t> done_at_;
    std::vector<Pending> pending_;
    int64_t base_;
    double per_unit_;
    int64_t fail_every_;
    int64_t t_ = 0, launches_ = 0, hazards_ = 0;
};

// The scheduler over a simulated device; arguments as checked by
// utf16wf_serve_simulate. *hazards counts launches given an arena region
// that work queued by a failed launch could still write.
inline int simulate(const utf16wf_serve_config &cfg, const int64_t *arrival_ns, const int64_t *lengths, int64_t n,
                    int64_t lat_base_ns, double lat_ns_per_unit, int64_t fail_every, utf16wf_serve_outcome *outcomes,
                    utf16wf_serve_stats *stats, int64_t *hazards) {
    std::vector<Request> rq((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        rq[(size_t)i] = Request{arrival_ns[i], lengths[i]};
    SimExec ex(cfg.num_streams, lat_base_ns, lat_ns_per_unit, fail_every);
    const int rc = run_loop(ex, cfg, rq.data(), n, outcomes, stats);
    *hazards = ex.hazards();
    return rc;
}

}  // namespace serve
}  // namespace utf16wf
