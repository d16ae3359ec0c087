// Host-only driver of the serving loop's scheduler (serve_core.h) over the
// simulated executor (serve_sim.h), built with AddressSanitizer and UBSan by
// tests/test_sanitizers.py. Random schedules, arenas, slot counts, batch
// limits, time-outs and injected launch failures; each run is checked for
// the scheduler's invariants and repeated to check that it is deterministic.
// Prints "ok" and exits 0, or names the first broken invariant and exits 1.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../paper_2601_06349_amd/csrc/serve_sim.h"

using namespace utf16wf::serve;

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
uint64_t next_u64() {  // xorshift64*
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return g_state * 0x2545F4914F6CDD1Dull;
}
int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }

int fail_case(int c, const char *what) {
    std::printf("case %d: %s\n", c, what);
    return 1;
}

bool same(const std::vector<utf16wf_serve_outcome> &a, const std::vector<utf16wf_serve_outcome> &b) {
    for (size_t i = 0; i < a.size(); ++i)
        if (a[i].launch_ns != b[i].launch_ns || a[i].done_ns != b[i].done_ns || a[i].status != b[i].status ||
            a[i].batch != b[i].batch || a[i].slot != b[i].slot)
            return false;
    return true;
}

}  // namespace

int main() {
    for (int c = 0; c < 200; ++c) {
        const int64_t n = uniform(0, 3000);
        std::vector<int64_t> arr(n), len(n);
        int64_t t = 0;
        for (int64_t i = 0; i < n; ++i) {
            t += uniform(0, 40000);
            arr[i] = t;
            const int64_t kind = uniform(0, 9);
            len[i] = kind == 0 ? 0 : kind < 7 ? uniform(1, 2000) : kind < 9 ? uniform(2000, 200000) : uniform(200000, 3000000);
        }
        utf16wf_serve_config cfg{};
        cfg.num_streams = (int32_t)uniform(1, 16);
        cfg.op = uniform(0, 1) ? UTF16WF_OP_TO : UTF16WF_OP_IS;
        cfg.arena_bytes = uniform(256, 8000000);
        cfg.max_batch_requests = uniform(1, 64);
        cfg.max_batch_units = uniform(1, 1 << 20);
        cfg.timeout_ns = uniform(0, 3) == 0 ? uniform(1, 5000000) : 0;
        cfg.separate_max = uniform(-1, 32);
        const int64_t fail_every = uniform(0, 2) == 0 ? 0 : uniform(1, 9);
        const int64_t base = uniform(0, 200000);
        const double per_unit = (double)uniform(0, 100) / 50.0;
        std::vector<utf16wf_serve_outcome> out(n), out2(n);
        utf16wf_serve_stats st{}, st2{};
        int64_t hz = 0, hz2 = 0;
        if (simulate(cfg, arr.data(), len.data(), n, base, per_unit, fail_every, out.data(), &st, &hz) != UTF16WF_OK)
            return fail_case(c, "simulate failed");
        if (hz != 0)
            return fail_case(c, "an arena region was reused while a failed launch's work could still write it");
        if (st.completed + st.rejected + st.timed_out + st.failed != n)
            return fail_case(c, "requests lost");
        if (st.arena_peak_bytes > cfg.arena_bytes)
            return fail_case(c, "arena budget exceeded");
        if (st.max_inflight > cfg.num_streams)
            return fail_case(c, "more batches in flight than slots");
        int32_t last_batch = -1;
        for (int64_t i = 0; i < n; ++i) {
            const utf16wf_serve_outcome &o = out[i];
            if (o.status != 0 && o.status != UTF16WF_ERANGE && o.status != UTF16WF_EHIP && o.status != kStatusTimedOut)
                return fail_case(c, "request left pending");
            if (o.status == 0 && (o.launch_ns < arr[i] || o.done_ns < o.launch_ns))
                return fail_case(c, "launched before arrival or done before launch");
            if (o.batch >= 0) {
                if (o.batch < last_batch)
                    return fail_case(c, "arrival order not kept");
                last_batch = o.batch;
            }
        }
        if (simulate(cfg, arr.data(), len.data(), n, base, per_unit, fail_every, out2.data(), &st2, &hz2) != UTF16WF_OK ||
            !same(out, out2) || st.batches != st2.batches || st.wall_ns != st2.wall_ns)
            return fail_case(c, "not deterministic");
    }
    std::printf("ok\n");
    return 0;
}
