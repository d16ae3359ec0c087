/*
 * utf16wf — UTF-16 well-formedness check and repair on one MI355X (gfx950).
 *
 * The operation (Clausecker & Lemire, "Fixing ill-formed UTF-16 strings with
 * SIMD instructions", arXiv 2601.06349):
 *   - 0xD800..0xDBFF is a high surrogate, 0xDC00..0xDFFF a low surrogate; a
 *     high immediately followed by a low is one supplementary character
 *     (Sec. 1, surrogate ranges and the code-point formula).
 *   - A high not followed by a low, or a low not preceded by a high, is
 *     mismatched; toWellFormed replaces each mismatched unit with U+FFFD and
 *     keeps the length (Sec. 1; Sec. 3.1, the per-unit blend with U+FFFD).
 *     isWellFormed reports whether no unit is mismatched (Sec. 3.1, the
 *     presence test over all blocks).
 *   - Before the first unit and after the last there is no surrogate, so a
 *     leading low and a trailing high are mismatched (Sec. 3.1, the two edge
 *     cases; Fig. 3 pads with U+0000).
 *   - Repair may run in place (output buffer = input buffer) or into a
 *     distinct buffer with the same result (Sec. 3).
 * Ragged batches (not in the paper): string k is units [off[k], off[k+1]) of
 * a packed buffer and is checked or repaired on its own; a high at the end of
 * one string never pairs with a low at the start of the next.
 *
 * Conventions for every call below:
 *   - Buffers are DEVICE memory on the current HIP device, allocated and owned
 *     by the caller; the library never frees them. Code units are host-order
 *     (little-endian) uint16. Lengths and offsets count code units.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream unless stated otherwise.
 *   - Return value: UTF16WF_OK (0) or a negative status. Argument checks
 *     (status -1..-4) all run before any HIP call and leave memory untouched.
 *     Content never causes an error: every uint16 sequence has a defined
 *     result.
 *   - utf16wf_last_error() returns a thread-local message for the last
 *     failure on the calling thread.
 */
#ifndef UTF16WF_H
#define UTF16WF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    UTF16WF_OK = 0,
    UTF16WF_EINVAL = -1,   /* null pointer with work to do, n < 0, num_strings < 0, bad op */
    UTF16WF_EALIGN = -2,   /* a uint16 pointer that is not 2-byte aligned, int64/int32 not 4/8 */
    UTF16WF_EOVERLAP = -3, /* input and output overlap without being equal */
    UTF16WF_EOFFSETS = -4, /* offsets not monotone or out of range (utf16wf_validate_offsets) */
    UTF16WF_EHIP = -5,     /* HIP runtime or launch failure; see utf16wf_last_error() */
    UTF16WF_ERANGE = -6,   /* request larger than a stated limit */
    UTF16WF_ENOMEM = -7    /* host or device allocation failed */
};

/* Operation codes for plans and tuning. */
enum {
    UTF16WF_OP_IS = 0,         /* isWellFormed                         */
    UTF16WF_OP_TO = 1,         /* toWellFormed into a distinct buffer  */
    UTF16WF_OP_TO_INPLACE = 2, /* toWellFormed in place                */
    UTF16WF_OP_LOCATE = 3      /* first mismatched index and count     */
};

/* ---------------------------------------------------------------- flat --- */

/* isWellFormed over in[0, n) (Sec. 3.1 presence test, closed at both ends).
 * Writes *result (device int32) = 1 if well-formed, else 0. n == 0 writes 1.
 * The kernel stops early once a mismatched unit has been seen. */
int utf16_is_well_formed(const uint16_t *in, int64_t n, int32_t *result, void *stream);

/* toWellFormed: out[0, n) = in[0, n) with every mismatched unit replaced by
 * U+FFFD (Sec. 1, Sec. 3.1). out == in runs in place (only the 128-byte
 * lines that hold a changed unit are written); any other overlap is
 * UTF16WF_EOVERLAP. Both pointers must be 2-byte aligned; any alignment runs
 * with 16-byte loads and stores except at the two ends, unless `in` and
 * `out` differ modulo 16 bytes: then the output is written unit by unit. */
int utf16_to_well_formed(const uint16_t *in, uint16_t *out, int64_t n, void *stream);

/* toWellFormed in place: same as utf16_to_well_formed(buf, buf, n, stream). */
int utf16_to_well_formed_inplace(uint16_t *buf, int64_t n, void *stream);

/* Locate (not in the paper's interface; the paper's presence test tells only
 * that a block holds a mismatch, Sec. 3.1 and Fig. 3): *first_bad = index of
 * the first mismatched unit or -1, *count = number of mismatched units (the
 * units toWellFormed would replace). Both outputs are device int64. */
int utf16_locate_ill_formed(const uint16_t *in, int64_t n, int64_t *first_bad, int64_t *count,
                            void *stream);

/* Host-resident input (not in the paper's interface; the paper's routine
 * repairs strings in the CPU's memory, Sec. 4): toWellFormed of h_in[0, n)
 * into h_out[0, n), both HOST memory (h_out == h_in repairs in place; any
 * other overlap is UTF16WF_EOVERLAP). The string moves through three device
 * staging slots in chunks of chunk_units (0 = 8 Mi units); each chunk is
 * copied in with one unit of context on each side, repaired, and its own
 * units copied back. Copies in run on one stream, repairs and copies out on
 * another, so both PCIe directions stay busy when the host buffers are
 * pinned (hipHostMalloc); pageable buffers work but are staged by the
 * runtime.
 * Synchronous: returns when h_out is complete. The staging buffer (up to
 * 256 MiB) and its streams are kept per device and reused by later calls;
 * a call that finds them in use, or needs more, uses private ones. */
int utf16_to_well_formed_host(const uint16_t *h_in, uint16_t *h_out, int64_t n, int64_t chunk_units);

/* -------------------------------------------------------- ragged batch --- */
/* offsets: device int64[num_strings + 1], non-decreasing, offsets[0] >= 0;
 * string k is units [offsets[k], offsets[k+1]) of the packed buffer. The
 * library trusts the offsets: callers that cannot guarantee them call
 * utf16wf_validate_offsets first. Units outside [offsets[0],
 * offsets[num_strings]) are neither read nor written. Empty strings are
 * well-formed. num_strings == 0 does nothing. */

/* results: device uint8[num_strings]; results[k] = 1 if string k is
 * well-formed, else 0. Tiles that lie inside a string already known to be
 * ill-formed are skipped. */
int utf16_is_well_formed_batch(const uint16_t *buf, const int64_t *offsets, int64_t num_strings,
                               uint8_t *results, void *stream);

/* toWellFormed per string into out, indexed by the same offsets (string k
 * goes to out[offsets[k], offsets[k+1])). out == in runs in place. Any other
 * overlap of in[offsets[0], offsets[B]) with out[offsets[0], offsets[B]) is
 * not allowed: the two ranges overlap exactly when in and out lie less than
 * offsets[B] - offsets[0] units apart. That span is only known on the
 * device, so this call cannot check it; utf16wf_batch with a size hint,
 * plan creation and utf16wf_validate_batch return UTF16WF_EOVERLAP for it. */
int utf16_to_well_formed_batch(const uint16_t *in, uint16_t *out, const int64_t *offsets,
                               int64_t num_strings, void *stream);

int utf16_to_well_formed_batch_inplace(uint16_t *buf, const int64_t *offsets, int64_t num_strings,
                                       void *stream);

/* Per string: first_bad[k] = index of the first mismatched unit relative to
 * offsets[k], or -1; count[k] = number of mismatched units. Device int64
 * arrays of num_strings entries. */
int utf16_locate_ill_formed_batch(const uint16_t *buf, const int64_t *offsets, int64_t num_strings,
                                  int64_t *first_bad, int64_t *count, void *stream);

/* General batch entry used by the ones above. op is a UTF16WF_OP_* code;
 * results is used by OP_IS; first_bad/count by OP_LOCATE (pass NULL
 * otherwise). units_hint, if > 0, is the caller's figure for
 * offsets[num_strings] - offsets[0]; it picks the tuned launch shape and
 * grid size and, for OP_IS, whether a head pass over long strings runs
 * first (0 = unknown: the shape for unknown sizes and a full persistent
 * grid). Any value gives the same results; a wrong one only costs speed.
 * OP_LOCATE over at most 256 strings takes the flat (batch 0) parameters of
 * that size class, the shape for one long string.
 * For UTF16WF_OP_TO with out != in and units_hint > 0, the hint is taken as
 * the span: buffers less than 2 * units_hint bytes apart are rejected with
 * UTF16WF_EOVERLAP before any HIP call. */
int utf16wf_batch(int op, const uint16_t *in, uint16_t *out, const int64_t *offsets,
                  int64_t num_strings, uint8_t *results, int64_t *first_bad, int64_t *count,
                  int64_t units_hint, void *stream);

/* Checks offsets on the device: non-decreasing, offsets[0] >= 0 and
 * offsets[num_strings] <= buf_units. Synchronous on `stream`. Returns
 * UTF16WF_OK or UTF16WF_EOFFSETS. Uses a small device workspace that the
 * library allocates on a device's first validation and keeps until the
 * process ends. */
int utf16wf_validate_offsets(const int64_t *offsets, int64_t num_strings, int64_t buf_units,
                             void *stream);

/* Everything a batch call trusts its caller for: the offsets as in
 * utf16wf_validate_offsets (UTF16WF_EOFFSETS), then, when out is neither
 * NULL nor in, that in[offsets[0], offsets[B]) and out[offsets[0],
 * offsets[B]) do not overlap (UTF16WF_EOVERLAP). Synchronous on `stream`;
 * the same workspace as utf16wf_validate_offsets. */
int utf16wf_validate_batch(const uint16_t *in, const uint16_t *out, const int64_t *offsets,
                           int64_t num_strings, int64_t buf_units, void *stream);

/* For callers that cannot allocate device memory (code in tight serving
 * loops, harnesses that forbid hipMalloc): utf16wf_validate_batch without
 * the workspace that it allocates on a device's first call. Its flag lives
 * in a 256-byte array of static device memory that every device the library
 * runs on holds until the process ends (the validation uses 4 bytes of it,
 * whatever the batch's size, so no batch is too large for it); the call
 * allocates nothing, neither device nor pinned memory. Same arguments,
 * checks, results and synchronisation as utf16wf_validate_batch. Every call
 * on one device shares that device's array, which keeps the last call's
 * contents (the flag is cleared by a kernel before each use): calls from
 * this process on one device are serialised by the library, while
 * validations that overlap on one device from several processes each use
 * their own process's array. */
int utf16wf_validate_batch_noalloc(const uint16_t *in, const uint16_t *out, const int64_t *offsets,
                                   int64_t num_strings, int64_t buf_units, void *stream);

/* ---------------------------------------------------------- batch plans --- */
/* A plan captures one batch call (its result initialisation and its
 * persistent kernel) into a HIP graph once; launching replays the graph on
 * `stream`. Buffers and num_strings are fixed at creation; their contents may
 * change between launches. The capture itself uses a private stream. At
 * creation the two ends of `offsets` are read on `stream` (which the call
 * synchronises; it must not be capturing) and the units they span size the
 * captured launch, as units_hint does for utf16wf_batch; offsets that change
 * later stay correct, the launch shape may only fit them less well. A
 * UTF16WF_OP_TO plan whose out and in overlap over that span is rejected
 * with UTF16WF_EOVERLAP. */
int utf16wf_batch_plan_create(int op, const uint16_t *in, uint16_t *out, const int64_t *offsets,
                              int64_t num_strings, uint8_t *results, void *stream, void **plan);
int utf16wf_batch_plan_launch(void *plan, void *stream);
int utf16wf_batch_plan_destroy(void *plan);

/* --------------------------------------------------------------- tuning --- */
/* Launch parameters of the kernels. rows: 16-byte loads in flight per lane
 * per tile (1, 2, 4 or 8; a tile is rows * 512 units per wave). wg_waves:
 * waves per workgroup (1..16). grid_per_cu: workgroups per compute unit of a
 * full persistent grid (1..64). nontemporal: 0/1, streaming cache hints.
 * store_lines: 0/1, the in-place repair's store mode (Sec. 3.2 writes only
 * where something changed): 1 writes every 128-byte line that holds a change
 * whole (the line's unchanged units written back as read), 0 writes only the
 * 16-byte vectors that changed; the other operations ignore it (default 1). */
typedef struct {
    int32_t rows;
    int32_t wg_waves;
    int32_t grid_per_cu;
    int32_t nontemporal;
    int32_t store_lines;
} utf16wf_params;

/* Set the parameters used for (op, batch 0/1, size class). size_class is
 * floor(log2(units)) in 0..40, or -1 for every class. */
int utf16wf_set_params(int op, int batch, int size_class, const utf16wf_params *p);
/* Parameters that a call of (op, batch, n units) would use: those set for
 * its size class; for a class with none set, those of the nearest class
 * that has some (the smaller on a tie); the built-in defaults when no class
 * of (op, batch) is set. */
int utf16wf_get_params(int op, int batch, int64_t n, utf16wf_params *p);
/* Back to the built-in defaults. */
int utf16wf_reset_params(void);

/* ---------------------------------------------------------- diagnostics --- */
/* Plain device copy of n uint16 units with the same tiling as the repair
 * kernels: the bandwidth ceiling that the repair is measured against. */
int utf16wf_copy_units(const uint16_t *in, uint16_t *out, int64_t n, void *stream);

/* Number of compute units of the current device (0 on failure). */
int utf16wf_device_cus(void);

/* Thread-local message of the last failing call. */
const char *utf16wf_last_error(void);
/* Version of this interface: 2 (utf16wf_params gained store_lines). */
int utf16wf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* UTF16WF_H */
