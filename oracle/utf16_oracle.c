/*
 * Scalar CPU oracle for UTF-16 well-formedness repair.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no code, header, table or helper with the
 * GPU path.
 *
 * What it computes (Clausecker & Lemire, "Fixing ill-formed UTF-16 strings
 * with SIMD instructions", arXiv 2601.06349):
 *   - A code unit in 0xD800..0xDBFF is a high surrogate and one in
 *     0xDC00..0xDFFF is a low surrogate; a character outside the BMP is a high
 *     surrogate immediately followed by a low surrogate (Sec. 1, the
 *     surrogate-pair ranges and the code-point formula).
 *   - A string is ill-formed when a high surrogate is not followed by a low
 *     one, or a low surrogate is not preceded by a high one (Sec. 1).
 *   - Repair replaces every such mismatched unit with U+FFFD and keeps the
 *     length unchanged (Abstract; Sec. 3.1, the blend step that writes U+FFFD
 *     over individual units of the block).
 *   - Positions before the first unit and after the last one hold no
 *     surrogate: a leading low and a trailing high are mismatched (Sec. 3.1,
 *     the two edge cases the vector procedure must handle by hand; Fig. 3
 *     pads the example with U+0000).
 *   - The result is the same whether the output buffer is the input buffer or
 *     a distinct one (Sec. 3, in-place and copy-based correction).
 *
 * The routines below are the plain sequential definition: walk the string
 * left to right, step over a high+low pair as one character, and replace any
 * other surrogate. No blocking, vectorisation or reordering. Build with
 * -O2 -fno-tree-vectorize so the loop stays scalar.
 *
 * Ragged batches (a packed buffer plus int64 offsets) are not in the paper;
 * the oracle applies the definition to each string [off[k], off[k+1]) on its
 * own, so no pair is formed across a string boundary.
 *
 * The chunked multi-threaded routine applies the same sequential walk to
 * contiguous chunks, reading at most one unit of context on each side of its
 * chunk. It exists only to time the oracle on several host cores.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define WF_REPLACEMENT 0xFFFDu

static int is_high(uint16_t u) { return u >= 0xD800u && u <= 0xDBFFu; }
static int is_low(uint16_t u) { return u >= 0xDC00u && u <= 0xDFFFu; }

/* Sequential walk over s[lo, hi) of a string of length n, writing replaced
 * units to t. Units of t outside [lo, hi) are not touched. A walk that starts
 * inside the string (lo > 0) first checks whether s[lo] is the low half of a
 * pair that starts at s[lo-1]; that is the only unit of left context it reads.
 * A pair starting at hi-1 reads s[hi] as right context. Returns the number of
 * units replaced in [lo, hi). */
static int64_t walk(const uint16_t *s, uint16_t *t, int64_t n, int64_t lo, int64_t hi)
{
    int64_t replaced = 0;
    int64_t i = lo;
    if (lo > 0 && lo < hi && is_low(s[lo]) && is_high(s[lo - 1]))
        i = lo + 1; /* s[lo] completes the pair that starts at s[lo-1] */
    while (i < hi) {
        uint16_t u = s[i];
        if (is_high(u) && i + 1 < n && is_low(s[i + 1])) {
            i += 2; /* a valid pair: one supplementary character */
        } else if (is_high(u) || is_low(u)) {
            t[i] = (uint16_t)WF_REPLACEMENT; /* a lone surrogate */
            replaced++;
            i += 1;
        } else {
            i += 1;
        }
    }
    return replaced;
}

/* toWellFormed, copy form: t[0..n) receives the repaired string. t may equal
 * s. Returns the number of units replaced. */
int64_t wf_to_seq(const uint16_t *s, uint16_t *t, int64_t n)
{
    if (n <= 0)
        return 0;
    if (t != s)
        memcpy(t, s, (size_t)n * sizeof(uint16_t));
    return walk(s, t, n, 0, n);
}

/* isWellFormed: 1 if no unit would be replaced, else 0. Stops at the first
 * lone surrogate. */
int wf_is_seq(const uint16_t *s, int64_t n)
{
    int64_t i = 0;
    while (i < n) {
        uint16_t u = s[i];
        if (is_high(u) && i + 1 < n && is_low(s[i + 1]))
            i += 2;
        else if (is_high(u) || is_low(u))
            return 0;
        else
            i += 1;
    }
    return 1;
}

/* Index of the first unit that toWellFormed would replace, or -1. */
int64_t wf_first_bad_seq(const uint16_t *s, int64_t n)
{
    int64_t i = 0;
    while (i < n) {
        uint16_t u = s[i];
        if (is_high(u) && i + 1 < n && is_low(s[i + 1]))
            i += 2;
        else if (is_high(u) || is_low(u))
            return i;
        else
            i += 1;
    }
    return -1;
}

/* Ragged batch, copy form: every string [off[k], off[k+1]) is repaired on its
 * own. Units of t outside [off[0], off[B]) are not touched. Returns the total
 * number of units replaced. */
int64_t wf_to_batch(const uint16_t *buf, uint16_t *t, const int64_t *off, int64_t num_strings)
{
    int64_t replaced = 0;
    for (int64_t k = 0; k < num_strings; k++) {
        int64_t a = off[k], len = off[k + 1] - off[k];
        replaced += wf_to_seq(buf + a, t + a, len);
    }
    return replaced;
}

/* Ragged batch isWellFormed: results[k] = 1 if string k is well-formed. */
void wf_is_batch(const uint16_t *buf, const int64_t *off, int64_t num_strings, uint8_t *results)
{
    for (int64_t k = 0; k < num_strings; k++)
        results[k] = (uint8_t)wf_is_seq(buf + off[k], off[k + 1] - off[k]);
}

/* Ragged batch: per-string count of replaced units and first replaced index
 * (relative to the string start, -1 if none). */
void wf_locate_batch(const uint16_t *buf, const int64_t *off, int64_t num_strings,
                     int64_t *first_bad, int64_t *count)
{
    for (int64_t k = 0; k < num_strings; k++) {
        const uint16_t *s = buf + off[k];
        int64_t n = off[k + 1] - off[k];
        first_bad[k] = wf_first_bad_seq(s, n);
        int64_t c = 0, i = 0;
        while (i < n) {
            uint16_t u = s[i];
            if (is_high(u) && i + 1 < n && is_low(s[i + 1]))
                i += 2;
            else {
                if (is_high(u) || is_low(u))
                    c++;
                i += 1;
            }
        }
        count[k] = c;
    }
}

/* ---- multi-threaded timing variant ------------------------------------- */

struct chunk_job {
    const uint16_t *s;
    uint16_t *t;
    int64_t n, lo, hi;
    int64_t replaced;
};

static void *chunk_main(void *arg)
{
    struct chunk_job *j = (struct chunk_job *)arg;
    if (j->t != j->s && j->hi > j->lo)
        memcpy(j->t + j->lo, j->s + j->lo, (size_t)(j->hi - j->lo) * sizeof(uint16_t));
    j->replaced = walk(j->s, j->t, j->n, j->lo, j->hi);
    return NULL;
}

/* toWellFormed on T threads over contiguous chunks. t must not equal s (each
 * chunk reads one unit of its neighbours' input). Returns units replaced, or
 * -1 if threads could not be created. */
int64_t wf_to_chunked_mt(const uint16_t *s, uint16_t *t, int64_t n, int threads)
{
    if (n <= 0)
        return 0;
    if (threads < 1)
        threads = 1;
    if ((int64_t)threads > n)
        threads = (int)n;
    struct chunk_job *jobs = calloc((size_t)threads, sizeof *jobs);
    pthread_t *tid = calloc((size_t)threads, sizeof *tid);
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return -1;
    }
    int64_t step = n / threads, started = 0, total = 0, failed = 0;
    for (int k = 0; k < threads; k++) {
        jobs[k].s = s;
        jobs[k].t = t;
        jobs[k].n = n;
        jobs[k].lo = (int64_t)k * step;
        jobs[k].hi = (k == threads - 1) ? n : (int64_t)(k + 1) * step;
        if (pthread_create(&tid[k], NULL, chunk_main, &jobs[k]) != 0) {
            failed = 1;
            break;
        }
        started++;
    }
    for (int64_t k = 0; k < started; k++) {
        pthread_join(tid[k], NULL);
        total += jobs[k].replaced;
    }
    free(jobs);
    free(tid);
    return failed ? -1 : total;
}
