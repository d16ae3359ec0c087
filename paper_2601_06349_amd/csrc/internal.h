// Host-side helpers of the library shared between the C entry points
// (api.cpp) and the serving loop (serve.cpp); not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace utf16wf {

// Records `msg` as the calling thread's last error and returns `code`.
int set_error(int code, const char *msg);

// Separate strings, at most kMultiMax, in one launch on `stream` (no
// packing; each string as a flat call of Sec. 1 / Sec. 3.1 semantics):
// string i is src[i][0, len[i]). op kOpTo writes its repair to dst[i]
// (dst[i] == src[i] repairs in place; other overlaps of a string's input
// and output are rejected). op kOpIs writes `stamp` to results[i] when
// string i is ill-formed and leaves the word alone otherwise (dst unused).
// Pointers are device pointers; every check runs before any HIP call.
// Returns UTF16WF_OK or a negative status.
int strings_call(int op, int n, const uint16_t *const *src, uint16_t *const *dst, const int64_t *len,
                 uint32_t *results, uint32_t stamp, hipStream_t stream);

// Batch validation as utf16wf_validate_batch does it, with the device int32
// `flag` supplied by the caller (who keeps other validations off it until
// the call returns): check_validate_batch_args makes the argument checks
// (no HIP call); validate_batch_with then checks the offsets on the device
// and the overlap of in and out over the span they give. Synchronous on s.
int check_validate_batch_args(const uint16_t *in, const uint16_t *out, const int64_t *offsets, int64_t nstr,
                              int64_t buf_units);
int validate_batch_with(const uint16_t *in, const uint16_t *out, const int64_t *offsets, int64_t nstr,
                        int64_t buf_units, hipStream_t s, int32_t *flag);

}  // namespace utf16wf
