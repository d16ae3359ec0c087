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

}  // namespace utf16wf
