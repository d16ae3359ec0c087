// Serving loop on the GPU (include/utf16wf_serve.h): the scheduler of
// serve_core.h driven by a HIP executor, and the same scheduler driven by the
// simulated executor of serve_sim.h (virtual clock, no GPU).
//
// HIP executor, per batch on its slot's stream (default priority).
// A batch of at most separate_max requests (at most kMultiMax) is one launch
// over the requests where they lie (each request a string of its own, its
// descriptors in the kernel's arguments): the repair goes straight to each
// destination, or to the batch's arena region for requests without one; the
// check stamps a per-slot result word. Larger batches are packed:
//   1. the batch's offsets and its gather / scatter descriptors, packed
//      together, in one copy from pinned host memory to the slot's device
//      staging buffer;
//   2. gather: each request's payload is copied into the packed input;
//   3. one batch launch (utf16wf_batch) repairs into the packed output, or
//      checks into per-string results;
//   4. scatter to the requests' destinations (if any).
// Then result bytes (the check) come back to pinned host memory, and an
// event follows; the loop polls it and then frees the region.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/utf16wf.h"
#include "../../include/utf16wf_serve.h"
#include "internal.h"
#include "kernels.h"
#include "serve_core.h"
#include "serve_sim.h"

using namespace utf16wf;
using namespace utf16wf::serve;

namespace {

int check_config(const utf16wf_serve_config *c, int64_t n) {
    if (!c)
        return set_error(UTF16WF_EINVAL, "null config");
    if (n < 0)
        return set_error(UTF16WF_EINVAL, "n < 0");
    if (c->num_streams < 1 || c->num_streams > 16)
        return set_error(UTF16WF_EINVAL, "num_streams must be 1..16");
    if (c->op != UTF16WF_OP_TO && c->op != UTF16WF_OP_IS)
        return set_error(UTF16WF_EINVAL, "op must be UTF16WF_OP_TO or UTF16WF_OP_IS");
    if (c->arena_bytes < 256 || c->max_batch_requests < 1 || c->max_batch_units < 1 || c->timeout_ns < 0)
        return set_error(UTF16WF_EINVAL, "bad arena / batch limits / timeout");
    if (c->separate_max < -1 || c->separate_max > kMultiMax)
        return set_error(UTF16WF_EINVAL, "separate_max must be -1..32");
    return UTF16WF_OK;
}

// ------------------------------------------------------------ HIP executor

class HipExec {
    struct Slot;

  public:
    HipExec(const utf16wf_serve_config &cfg, const utf16wf_serve_request *reqs, int64_t n)
        : cfg_(cfg), reqs_(reqs), n_(n), separate_max_(cfg.separate_max == 0 ? kMultiMax : cfg.separate_max) {}

    int init() {
        int64_t max_len = 0;
        for (int64_t i = 0; i < n_; ++i)
            max_len = std::max(max_len, reqs_[i].length);
        const int64_t cap_units = std::max(cfg_.max_batch_units, max_len);
        const int64_t cap_req = std::min<int64_t>(cfg_.max_batch_requests, std::max<int64_t>(n_, 1));
        max_chunks_ = cap_units / kCopyChunkUnits + cap_req + 1;
        max_req_ = cap_req;
        hipError_t e = hipMalloc(&arena_, (size_t)cfg_.arena_bytes);
        if (e != hipSuccess)
            return fail(e, "hipMalloc(arena)");
        const int slots = cfg_.num_streams;
        slot_.resize(slots);
        for (int s = 0; s < slots; ++s) {
            Slot &sl = slot_[s];
            if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess)
                return fail(e, "hipStreamCreateWithFlags");
            if ((e = hipEventCreateWithFlags(&sl.event, hipEventDisableTiming)) != hipSuccess)
                return fail(e, "hipEventCreateWithFlags");
            const size_t stage = 8 * (size_t)(max_req_ + 1) + 2 * sizeof(CopyChunk) * (size_t)max_chunks_;
            if ((e = hipHostMalloc((void **)&sl.h_stage, stage, 0)) != hipSuccess ||
                (e = hipHostMalloc((void **)&sl.h_res, max_req_ + 1, 0)) != hipSuccess)
                return fail(e, "hipHostMalloc");
            if ((e = hipMalloc((void **)&sl.d_stage, stage)) != hipSuccess)
                return fail(e, "hipMalloc(staging)");
            // result words of batches launched as separate strings: zero,
            // and stamps start at 1
            if ((e = hipMalloc((void **)&sl.d_words, 4 * kMultiMax)) != hipSuccess ||
                (e = hipHostMalloc((void **)&sl.h_words, 4 * kMultiMax, 0)) != hipSuccess)
                return fail(e, "result words");
            if ((e = hipMemset(sl.d_words, 0, 4 * kMultiMax)) != hipSuccess)
                return fail(e, "hipMemset(result words)");
        }
        t0_ = std::chrono::steady_clock::now();
        return UTF16WF_OK;
    }

    ~HipExec() {
        for (Slot &sl : slot_) {
            if (sl.stream)
                (void)hipStreamSynchronize(sl.stream);
        }
        for (Slot &sl : slot_) {
            if (sl.event)
                (void)hipEventDestroy(sl.event);
            if (sl.stream)
                (void)hipStreamDestroy(sl.stream);
            if (sl.h_stage)
                (void)hipHostFree(sl.h_stage);
            if (sl.h_res)
                (void)hipHostFree(sl.h_res);
            if (sl.d_stage)
                (void)hipFree(sl.d_stage);
            if (sl.d_words)
                (void)hipFree(sl.d_words);
            if (sl.h_words)
                (void)hipHostFree(sl.h_words);
        }
        if (arena_)
            (void)hipFree(arena_);
    }

    int64_t now() const {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0_).count();
    }

    int launch(Batch &b) {
        Slot &sl = slot_[b.slot];
        uint8_t *base = static_cast<uint8_t *>(arena_) + b.region;
        uint16_t *d_in = reinterpret_cast<uint16_t *>(base + b.lay.in_off);
        uint16_t *d_out = reinterpret_cast<uint16_t *>(base + b.lay.out_off);
        uint8_t *d_res = base + b.lay.results_off;
        const int64_t nb = (int64_t)b.reqs.size();
        sl.direct = nb <= separate_max_;
        if (sl.direct)
            return launch_direct(b, sl, d_out);
        // count the copy pieces first, so offsets, gather and scatter
        // descriptors lie back to back in the staging buffer
        int64_t g = 0, sc = 0;
        for (int64_t i = 0; i < nb; ++i) {
            const utf16wf_serve_request &r = reqs_[b.reqs[i]];
            const int64_t pieces = (r.length + kCopyChunkUnits - 1) / kCopyChunkUnits;
            g += pieces;
            if (r.dst && cfg_.op == UTF16WF_OP_TO)
                sc += pieces;
        }
        int64_t *h_off = reinterpret_cast<int64_t *>(sl.h_stage);
        CopyChunk *gat = reinterpret_cast<CopyChunk *>(sl.h_stage + 8 * (nb + 1));
        CopyChunk *sca = gat + g;
        int64_t gi = 0, si = 0, pos = 0;
        h_off[0] = 0;
        for (int64_t i = 0; i < nb; ++i) {
            const utf16wf_serve_request &r = reqs_[b.reqs[i]];
            for (int64_t c = 0; c < r.length; c += kCopyChunkUnits) {
                const int64_t len = std::min(kCopyChunkUnits, r.length - c);
                gat[gi++] = CopyChunk{r.src + c, d_in + pos + c, len};
                if (r.dst && cfg_.op == UTF16WF_OP_TO)
                    sca[si++] = CopyChunk{d_out + pos + c, r.dst + c, len};
            }
            pos += r.length;
            h_off[i + 1] = pos;
        }
        const size_t stage_bytes = 8 * (size_t)(nb + 1) + sizeof(CopyChunk) * (size_t)(g + sc);
        int64_t *d_offs = reinterpret_cast<int64_t *>(sl.d_stage);
        const CopyChunk *d_gat = reinterpret_cast<const CopyChunk *>(sl.d_stage + 8 * (nb + 1));
        hipStream_t st = sl.stream;
        hipError_t e;
        if ((e = hipMemcpyAsync(sl.d_stage, sl.h_stage, stage_bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
            return fail(e, "copy offsets and descriptors");
        if ((e = launch_chunk_copy(d_gat, g, st)) != hipSuccess)
            return fail(e, "gather");
        int rc;
        if (cfg_.op == UTF16WF_OP_TO)
            rc = utf16wf_batch(UTF16WF_OP_TO, d_in, d_out, d_offs, nb, nullptr, nullptr, nullptr, pos, st);
        else
            rc = utf16wf_batch(UTF16WF_OP_IS, d_in, nullptr, d_offs, nb, d_res, nullptr, nullptr, pos, st);
        if (rc != UTF16WF_OK)
            return rc;
        if (sc > 0 && (e = launch_chunk_copy(d_gat + g, sc, st)) != hipSuccess)
            return fail(e, "scatter");
        if (cfg_.op == UTF16WF_OP_IS &&
            (e = hipMemcpyAsync(sl.h_res, d_res, nb, hipMemcpyDeviceToHost, st)) != hipSuccess)
            return fail(e, "copy results");
        if ((e = hipEventRecord(sl.event, st)) != hipSuccess)
            return fail(e, "hipEventRecord");
        return UTF16WF_OK;
    }

    // The batch as separate strings: one launch, no copies of the payloads.
    int launch_direct(const Batch &b, Slot &sl, uint16_t *d_out) {
        const int n = (int)b.reqs.size();
        const uint16_t *src[kMultiMax];
        uint16_t *dst[kMultiMax];
        int64_t len[kMultiMax];
        int64_t pos = 0;
        for (int i = 0; i < n; ++i) {
            const utf16wf_serve_request &r = reqs_[b.reqs[i]];
            src[i] = r.src;
            len[i] = r.length;
            dst[i] = r.dst;
            if (!r.dst) {
                // into the arena region, at the input's phase (mod 8 units),
                // so whole 16-byte vectors are stored; the layout reserves
                // the 7 units this may skip per request
                pos += (int64_t)(((reinterpret_cast<uintptr_t>(r.src) >> 1) - (uintptr_t)pos) & 7u);
                dst[i] = d_out + pos;
                pos += r.length;
            }
        }
        hipStream_t st = sl.stream;
        int rc;
        hipError_t e;
        if (cfg_.op == UTF16WF_OP_TO) {
            rc = strings_call(kOpTo, n, src, dst, len, nullptr, 0u, st);
        } else {
            sl.stamp = (uint32_t)(b.id + 1);  // never 0, the words' initial value, before 2^32 batches
            rc = strings_call(kOpIs, n, src, nullptr, len, sl.d_words, sl.stamp, st);
            if (rc == UTF16WF_OK &&
                (e = hipMemcpyAsync(sl.h_words, sl.d_words, 4 * (size_t)n, hipMemcpyDeviceToHost, st)) != hipSuccess)
                return fail(e, "copy result words");
        }
        if (rc != UTF16WF_OK)
            return rc;
        if ((e = hipEventRecord(sl.event, st)) != hipSuccess)
            return fail(e, "hipEventRecord");
        ++direct_batches_;
        return UTF16WF_OK;
    }

    int64_t direct_batches() const { return direct_batches_; }

    int done(int slot) {
        const hipError_t e = hipEventQuery(slot_[slot].event);
        if (e == hipSuccess)
            return 1;
        if (e == hipErrorNotReady)
            return 0;
        fail(e, "hipEventQuery");
        return -1;
    }

    void drain(int slot) { (void)hipStreamSynchronize(slot_[slot].stream); }

    void finish(const Batch &b, utf16wf_serve_outcome *out) {
        if (cfg_.op != UTF16WF_OP_IS)
            return;
        const Slot &sl = slot_[b.slot];
        for (size_t i = 0; i < b.reqs.size(); ++i)
            out[b.reqs[i]].well_formed = sl.direct ? (sl.h_words[i] != sl.stamp ? 1 : 0) : sl.h_res[i];
    }

    void idle(int64_t next_arrival, bool any_busy) {
        if (any_busy) {
            std::this_thread::yield();
            return;
        }
        if (next_arrival < 0)
            return;
        const int64_t wait = next_arrival - now();
        if (wait > 200000)
            std::this_thread::sleep_for(std::chrono::nanoseconds(wait - 100000));
    }

  private:
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t event = nullptr;
        uint8_t *h_stage = nullptr;  // pinned: offsets, gather and scatter descriptors
        uint8_t *h_res = nullptr;
        uint8_t *d_stage = nullptr;  // device copy of h_stage
        uint32_t *d_words = nullptr; // check results of a separate-strings batch
        uint32_t *h_words = nullptr; // (pinned copy)
        uint32_t stamp = 0;          // the stamp of the slot's last such batch
        bool direct = false;         // the slot's batch runs as separate strings
    };
    int fail(hipError_t e, const char *where) {
        char buf[256];
        snprintf(buf, sizeof buf, "serve: %s: %s", where, hipGetErrorString(e));
        return set_error(UTF16WF_EHIP, buf);
    }

    utf16wf_serve_config cfg_;
    const utf16wf_serve_request *reqs_;
    int64_t n_;
    int64_t max_chunks_ = 0, max_req_ = 0, direct_batches_ = 0;
    int64_t separate_max_;  // batches of at most this many requests: separate strings (-1: none)
    void *arena_ = nullptr;
    std::vector<Slot> slot_;
    std::chrono::steady_clock::time_point t0_;
};

}  // namespace

extern "C" {

int utf16wf_serve_run(const utf16wf_serve_config *cfg, const utf16wf_serve_request *reqs, int64_t n,
                      utf16wf_serve_outcome *outcomes, utf16wf_serve_stats *stats) {
    int rc = check_config(cfg, n);
    if (rc != UTF16WF_OK)
        return rc;
    if (n > 0 && (!reqs || !outcomes))
        return set_error(UTF16WF_EINVAL, "null requests or outcomes");
    std::vector<Request> rq((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        if (reqs[i].length < 0 || (reqs[i].length > 0 && !reqs[i].src))
            return set_error(UTF16WF_EINVAL, "request with negative length or null payload");
        if (reinterpret_cast<uintptr_t>(reqs[i].src) & 1u || reinterpret_cast<uintptr_t>(reqs[i].dst) & 1u)
            return set_error(UTF16WF_EALIGN, "request pointer not 2-byte aligned");
        if (i > 0 && reqs[i].arrival_ns < reqs[i - 1].arrival_ns)
            return set_error(UTF16WF_EINVAL, "arrivals must be non-decreasing");
        const uintptr_t s = reinterpret_cast<uintptr_t>(reqs[i].src), d = reinterpret_cast<uintptr_t>(reqs[i].dst);
        const uintptr_t bytes = 2u * (uintptr_t)reqs[i].length;
        if (reqs[i].dst && s != d && s < d + bytes && d < s + bytes)
            return set_error(UTF16WF_EOVERLAP, "request destination overlaps its payload without being equal");
        rq[(size_t)i] = Request{reqs[i].arrival_ns, reqs[i].length};
    }
    HipExec ex(*cfg, reqs, n);
    if ((rc = ex.init()) != UTF16WF_OK)
        return rc;
    rc = run_loop(ex, *cfg, rq.data(), n, outcomes, stats);
    if (stats)
        stats->direct_batches = ex.direct_batches();
    return rc;
}

int utf16wf_serve_simulate(const utf16wf_serve_config *cfg, const int64_t *arrival_ns, const int64_t *lengths,
                           int64_t n, int64_t lat_base_ns, double lat_ns_per_unit, int64_t fail_every,
                           utf16wf_serve_outcome *outcomes, utf16wf_serve_stats *stats) {
    int rc = check_config(cfg, n);
    if (rc != UTF16WF_OK)
        return rc;
    if (n > 0 && (!arrival_ns || !lengths || !outcomes))
        return set_error(UTF16WF_EINVAL, "null arrays");
    if (lat_base_ns < 0 || lat_ns_per_unit < 0 || fail_every < 0)
        return set_error(UTF16WF_EINVAL, "negative latency model");
    for (int64_t i = 0; i < n; ++i)
        if (lengths[i] < 0 || (i > 0 && arrival_ns[i] < arrival_ns[i - 1]))
            return set_error(UTF16WF_EINVAL, "negative length or decreasing arrivals");
    int64_t hazards = 0;
    rc = simulate(*cfg, arrival_ns, lengths, n, lat_base_ns, lat_ns_per_unit, fail_every, outcomes, stats, &hazards);
    if (rc == UTF16WF_OK && hazards > 0) {
        char buf[160];
        snprintf(buf, sizeof buf, "simulation: %lld launches got an arena region that work queued by a failed launch "
                 "could still write", (long long)hazards);
        return set_error(UTF16WF_EHIP, buf);
    }
    return rc;
}

}  // extern "C"
