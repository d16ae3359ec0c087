/*
 * utf16wf serving loop: continuous batching of UTF-16 repair requests on one
 * GPU. Not part of the paper (whose routine is a library call, Sec. 3); each
 * request is repaired or checked alone, with the semantics of Sec. 1 and
 * Sec. 3.1, by the library's kernels for separate strings or for ragged
 * batches (utf16wf.h).
 *
 * Requests arrive on a schedule (arrival times relative to the start of the
 * run). A request is admitted when the arena (one device allocation, the HBM
 * budget) has room for its batch's region and a stream slot is free; batches
 * on different slots run concurrently, and requests that arrive while
 * batches are on the GPU join the next batch as soon as a slot and memory
 * free up. Requests are admitted in arrival order (no reordering).
 *
 * A batch of at most 32 requests (separate_max) is one launch over the
 * requests where they lie, each a string of its own: the repair goes
 * straight from the payload to the destination (or into the batch's arena
 * region when the request has none). A larger batch is packed: each payload is copied into the batch's
 * arena region, one ragged-batch launch repairs (or checks) it there, and
 * requests with a destination are copied out. Either way every request is
 * repaired alone, as one string.
 *
 * Payloads and destinations of requests that may be in flight together must
 * not overlap one another (a destination equal to its own payload is
 * allowed: in place).
 *
 * Conventions as in utf16wf.h: device pointers, return UTF16WF_OK or a
 * negative status, utf16wf_last_error() for the message.
 */
#ifndef UTF16WF_SERVE_H
#define UTF16WF_SERVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t num_streams;        /* batches in flight at once, 1..16 */
    int32_t op;                 /* UTF16WF_OP_TO (repair) or UTF16WF_OP_IS (check) */
    int64_t arena_bytes;        /* HBM budget: one device arena of this size */
    int64_t max_batch_requests; /* at most this many requests per batch (>= 1) */
    int64_t max_batch_units;    /* a batch stops growing past this many units (>= 1) */
    int64_t timeout_ns;         /* a request still waiting this long after its
                                   arrival is dropped (0 = never) */
    int64_t separate_max;       /* batches of at most this many requests run as
                                   separate strings, larger ones packed: 0 = 32
                                   (the most), 1..32, or -1 = always packed */
} utf16wf_serve_config;

typedef struct {
    int64_t arrival_ns;  /* scheduled arrival, non-decreasing over the array */
    const uint16_t *src; /* device payload (any 2-byte alignment) */
    int64_t length;      /* units, >= 0 */
    uint16_t *dst;       /* device destination for the repaired units, or NULL */
} utf16wf_serve_request;

typedef struct {
    int64_t launch_ns;   /* when its batch was launched (-1 if never) */
    int64_t done_ns;     /* when the host saw its batch complete (-1 if never) */
    int32_t status;      /* 0 done; UTF16WF_ERANGE larger than the arena;
                            UTF16WF_EHIP launch failure; 1 timed out */
    int32_t batch;       /* batch index modulo 2^31 (-1 if never launched) */
    int32_t slot;        /* stream slot of its batch */
    int32_t well_formed; /* UTF16WF_OP_IS: 1 / 0; otherwise -1 */
} utf16wf_serve_outcome;

typedef struct {
    int64_t batches;
    int64_t completed;
    int64_t rejected;          /* larger than the whole arena */
    int64_t timed_out;
    int64_t failed;            /* batch launch failed */
    int64_t max_inflight;      /* most batches in flight at once */
    int64_t max_queue;         /* most requests waiting for admission */
    int64_t arena_peak_bytes;  /* most arena bytes in use at once */
    int64_t wall_ns;           /* from start to the last completion */
    int64_t direct_batches;    /* batches launched as separate strings (no packing) */
} utf16wf_serve_stats;

/* Runs the loop on the current device until every request is completed,
 * rejected or timed out. Allocates the arena and per-slot buffers at the
 * start and frees them at the end. Outcomes has n entries. Synchronous.
 * Before any HIP call, returns UTF16WF_EINVAL for a bad configuration, a
 * negative length, a null payload or decreasing arrivals, UTF16WF_EALIGN
 * for a pointer that is not 2-byte aligned, and UTF16WF_EOVERLAP for a
 * destination that overlaps its own payload without being equal to it. */
int utf16wf_serve_run(const utf16wf_serve_config *cfg, const utf16wf_serve_request *reqs, int64_t n,
                      utf16wf_serve_outcome *outcomes, utf16wf_serve_stats *stats);

/* The same scheduler with a simulated executor and a virtual clock, no GPU:
 * a batch of U units completes lat_base_ns + lat_ns_per_unit * U after its
 * launch; if fail_every > 0, every fail_every-th batch fails at launch, after
 * its work was queued (that work still occupies its arena region until it
 * would have completed). For capacity planning and for testing the scheduler
 * on a CPU. Returns UTF16WF_EHIP if the scheduler ever gave a batch an arena
 * region that such queued work could still write. */
int utf16wf_serve_simulate(const utf16wf_serve_config *cfg, const int64_t *arrival_ns, const int64_t *lengths,
                           int64_t n, int64_t lat_base_ns, double lat_ns_per_unit, int64_t fail_every,
                           utf16wf_serve_outcome *outcomes, utf16wf_serve_stats *stats);

#ifdef __cplusplus
}
#endif

#endif /* UTF16WF_SERVE_H */
