// Internal interface between the host dispatcher (api.cpp) and the device
// kernels (kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace utf16wf {

enum Op : int { kOpIs = 0, kOpTo = 1, kOpToInplace = 2, kOpLocate = 3 };

struct LaunchShape {
    int rows;         // 1, 2, 4 or 8 sixteen-byte loads per lane per tile
    int wg_waves;     // waves per workgroup, 1..16
    int grid;         // workgroups
    int nontemporal;  // 0/1
    int store_lines;  // in-place repair: 1 whole 128-byte lines, 0 changed 16-byte vectors
};

// One launch of the repair/check kernel.
//  in, out      frame base pointers (16-byte aligned for `in`); unit u of the
//               frame is in[u] / out[u]
//  lo, hi       valid frame units [lo, hi) (flat calls; batch calls read them
//               from offsets)
//  offsets      batch: device int64[nstr + 1]; flat: nullptr
//  shift        batch: frame unit of buffer unit 0 (0..7)
//  flag         flat OP_IS: device int32 result (pre-set to 1)
//  results      batch OP_IS: device uint8[nstr] (pre-set to 1)
//  first, count OP_LOCATE: device int64 (pre-set to -1 and 0)
//  scalar_store store unit by unit (output phase differs from input phase)
struct KernelArgs {
    const uint16_t *in;
    uint16_t *out;
    int64_t lo, hi;
    const int64_t *offsets;
    int64_t nstr;
    int32_t shift;
    int32_t *flag;
    uint8_t *results;
    int64_t *first;
    int64_t *count;
    int scalar_store;
};

hipError_t launch_main(int op, bool batch, const LaunchShape &shape, const KernelArgs &a,
                       hipStream_t stream);
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t stream);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t stream);
// first[0, n) = -1 and count[0, n) = 0 in one launch (locate results).
hipError_t launch_fill_locate(int64_t *first, int64_t *count, int64_t n, hipStream_t stream);
hipError_t launch_copy(const uint16_t *in, uint16_t *out, int64_t lo, int64_t hi,
                       const LaunchShape &shape, hipStream_t stream);
// One contiguous piece of a gather or scatter copy (at most kCopyChunkUnits).
struct CopyChunk {
    const uint16_t *src;
    uint16_t *dst;
    int64_t n;
};
constexpr int64_t kCopyChunkUnits = 16384;
hipError_t launch_chunk_copy(const CopyChunk *chunks, int64_t nchunks, hipStream_t stream);

// Up to kMultiMax separate strings in one launch, each read from and written
// to its own place (no packing into one buffer). Each string is tiled alone,
// as the frame of a flat call: `in` / `out` are frame bases (unit u at in[u] /
// out[u]; `in` 16-byte aligned), the string is units [lo, hi) of its frame.
// Tiles are numbered string after string from 0 (`tile0` = the number of the
// string's first tile, `ntiles` in all); the kernel's rows per tile fix the
// tile size, so tile0 must be computed for the same rows.
// Repair (kOpTo) writes every unit of every string; `scalar_store` marks a
// string whose output phase (address mod 16) differs from its input's.
// Check (kOpIs) writes `stamp` to results[i] when string i has a mismatch and
// nothing otherwise: a string is well-formed iff its word differs from the
// stamp afterwards, so the words need no clearing between launches as long
// as every launch uses a new stamp.
constexpr int kMultiMax = 32;
struct MultiString {
    const uint16_t *in;
    uint16_t *out;
    int64_t lo, hi;
    int64_t tile0;
    int32_t scalar_store;
    int32_t pad_;
};
struct MultiArgs {
    MultiString s[kMultiMax];
    int64_t ntiles;
    uint32_t *results;
    int32_t n;
    uint32_t stamp;
};
hipError_t launch_multi(int op, const LaunchShape &shape, const MultiArgs &a, hipStream_t stream);

// Batch isWellFormed of few long strings, before the main pass: sets every
// string's result, 0 for a string of at least 8192 units with a mismatch
// among its first 512 units, else 1.
hipError_t launch_head_check(const uint16_t *in_frame, const int64_t *offsets, int64_t nstr, int64_t shift,
                             uint8_t *results, hipStream_t stream);

hipError_t launch_validate(const int64_t *offsets, int64_t nstr, int64_t buf_units, int32_t *bad,
                           hipStream_t stream);

}  // namespace utf16wf
