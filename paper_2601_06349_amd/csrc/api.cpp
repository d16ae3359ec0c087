// Host side of the C ABI declared in include/utf16wf.h: argument checks,
// launch-shape selection (tuned parameters per operation and size class),
// result initialisation, batch plans captured into HIP graphs, and the
// thread-local error message.
//
// Every argument check runs before the first HIP call, so a rejected call
// touches neither memory nor the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/utf16wf.h"
#include "internal.h"
#include "kernels.h"

using namespace utf16wf;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *where) {
    return fail(UTF16WF_EHIP, "%s: %s", where, hipGetErrorString(e));
}

// ---------------------------------------------------------- device info

constexpr int kMaxDevices = 64;
std::atomic<int> g_cus[kMaxDevices];

int current_device(int *dev) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    if (*dev < 0 || *dev >= kMaxDevices)
        return fail(UTF16WF_EHIP, "device ordinal %d out of range", *dev);
    return UTF16WF_OK;
}

int device_cus(int dev, int *cus) {
    int c = g_cus[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        hipError_t e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess)
            return hip_fail(e, "hipDeviceGetAttribute");
        if (c <= 0)
            c = 1;
        g_cus[dev].store(c, std::memory_order_relaxed);
    }
    *cus = c;
    return UTF16WF_OK;
}

// ------------------------------------------------------------ parameters

constexpr int kOps = 4;
constexpr int kClasses = 41;
std::mutex g_param_mu;
// batch OP_LOCATE over at most this many strings takes the flat parameters
constexpr int64_t kLocateFlatShapeMax = 256;

utf16wf_params g_params[kOps][2][kClasses];
bool g_params_set[kOps][2][kClasses];  // set by utf16wf_set_params (tuned)
bool g_params_init = false;

utf16wf_params default_params(int op, int batch, int cls) {
    utf16wf_params p;
    // Small inputs: short tiles so that enough waves exist to spread over
    // every compute unit; large inputs: four 16-byte loads in flight per
    // lane and a full persistent grid.
    p.rows = (batch || cls >= 22) ? 4 : (cls >= 20 ? 2 : 1);
    p.wg_waves = 4;
    p.grid_per_cu = 8;
    p.nontemporal = 0;
    p.store_lines = 1;
    (void)op;
    return p;
}

void init_params_locked() {
    if (g_params_init)
        return;
    for (int o = 0; o < kOps; ++o)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < kClasses; ++c) {
                g_params[o][b][c] = default_params(o, b, c);
                g_params_set[o][b][c] = false;
            }
    g_params_init = true;
}

int size_class(int64_t n) {
    int c = 0;
    while (c < kClasses - 1 && (n >> (c + 1)) > 0)
        ++c;
    return c;
}

bool params_ok(const utf16wf_params &p) {
    const bool rows_ok = p.rows == 1 || p.rows == 2 || p.rows == 4 || p.rows == 8;
    return rows_ok && p.wg_waves >= 1 && p.wg_waves <= 16 && p.grid_per_cu >= 1 && p.grid_per_cu <= 64 &&
           (p.nontemporal == 0 || p.nontemporal == 1) && (p.store_lines == 0 || p.store_lines == 1);
}

// The parameters set for n's size class; for a class that has none, those
// of the nearest class that has (the smaller on a tie), so sizes beyond the
// tuned range keep a tuned shape; the built-in defaults if none is set.
utf16wf_params get_params(int op, int batch, int64_t n) {
    std::lock_guard<std::mutex> lk(g_param_mu);
    init_params_locked();
    const int b = batch ? 1 : 0, c = size_class(n);
    for (int d = 0; d < kClasses; ++d) {
        if (c - d >= 0 && g_params_set[op][b][c - d])
            return g_params[op][b][c - d];
        if (c + d < kClasses && g_params_set[op][b][c + d])
            return g_params[op][b][c + d];
    }
    return g_params[op][b][c];
}

// Launch shape for a flat call over frame units [lo, hi), or for a batch with
// `units` (0 = unknown) units.
LaunchShape make_shape(const utf16wf_params &p, int cus, int64_t units, int64_t first_unit) {
    LaunchShape s;
    s.rows = p.rows;
    s.wg_waves = p.wg_waves;
    s.nontemporal = p.nontemporal;
    s.store_lines = p.store_lines;
    const int64_t max_waves = (int64_t)p.grid_per_cu * cus * p.wg_waves;
    int64_t waves = max_waves;
    if (units > 0) {
        const int64_t T = 512LL * p.rows;
        const int64_t tiles = (first_unit % T + units + T - 1) / T + 1;
        waves = std::min<int64_t>(tiles, max_waves);
    }
    s.grid = (int)std::max<int64_t>(1, (waves + p.wg_waves - 1) / p.wg_waves);
    return s;
}

// --------------------------------------------------------- workspace

struct Workspace {
    int32_t *flag = nullptr;
};
std::mutex g_ws_mu;
Workspace g_ws[kMaxDevices];
std::mutex g_validate_mu[kMaxDevices];

// Host-resident repair: staging buffer, streams and events kept per device
// between calls (at most kHostStagingCacheBytes; held until the process ends).
constexpr int kHostStages = 3;
constexpr size_t kHostStagingCacheBytes = (size_t)256 << 20;
struct HostStaging {
    std::mutex mu;
    uint16_t *buf = nullptr;
    size_t bytes = 0;
    hipStream_t in = nullptr, out = nullptr;
    hipEvent_t loaded[kHostStages] = {}, freed[kHostStages] = {};

    int ensure_streams() {
        hipError_t e;
        if (!in && (e = hipStreamCreateWithFlags(&in, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreateWithFlags");
        if (!out && (e = hipStreamCreateWithFlags(&out, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreateWithFlags");
        for (int i = 0; i < kHostStages; ++i) {
            if (!loaded[i] && (e = hipEventCreateWithFlags(&loaded[i], hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "hipEventCreateWithFlags");
            if (!freed[i] && (e = hipEventCreateWithFlags(&freed[i], hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "hipEventCreateWithFlags");
        }
        return UTF16WF_OK;
    }
    void release() {
        for (int i = 0; i < kHostStages; ++i) {
            if (loaded[i])
                (void)hipEventDestroy(loaded[i]);
            if (freed[i])
                (void)hipEventDestroy(freed[i]);
        }
        if (in)
            (void)hipStreamDestroy(in);
        if (out)
            (void)hipStreamDestroy(out);
        if (buf)
            (void)hipFree(buf);
    }
};
HostStaging g_host_staging[kMaxDevices];

int workspace(int dev, Workspace **ws) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (!g_ws[dev].flag) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, 256);
        if (e != hipSuccess)
            return hip_fail(e, "hipMalloc(workspace)");
        g_ws[dev].flag = static_cast<int32_t *>(p);
    }
    *ws = &g_ws[dev];
    return UTF16WF_OK;
}

// ---------------------------------------------------------- helpers

inline uintptr_t addr(const void *p) { return reinterpret_cast<uintptr_t>(p); }

bool overlap_not_equal(const void *a, const void *b, int64_t n_units) {
    if (a == b || n_units <= 0)
        return false;
    const uintptr_t x = addr(a), y = addr(b), len = (uintptr_t)n_units * 2u;
    return x < y + len && y < x + len;
}

int check_op(int op) {
    if (op < 0 || op >= kOps)
        return fail(UTF16WF_EINVAL, "unknown op %d", op);
    return UTF16WF_OK;
}

// Flat entry shared by is / to / to_inplace / locate.
int flat_call(int op, const uint16_t *in, uint16_t *out, int64_t n, int32_t *flag, int64_t *first,
              int64_t *count, hipStream_t stream) {
    int dev, cus, rc;
    if ((rc = current_device(&dev)) != UTF16WF_OK)
        return rc;
    if ((rc = device_cus(dev, &cus)) != UTF16WF_OK)
        return rc;
    hipError_t e;
    if (op == kOpIs) {
        if ((e = launch_fill_i32(flag, 1, 1, stream)) != hipSuccess)
            return hip_fail(e, "fill result");
    } else if (op == kOpLocate) {
        if ((e = launch_fill_locate(first, count, 1, stream)) != hipSuccess)
            return hip_fail(e, "fill first_bad and count");
    }
    if (n == 0)
        return UTF16WF_OK;
    const int64_t m = (int64_t)((addr(in) & 15u) >> 1);
    KernelArgs a{};
    a.in = in - m;
    a.out = out ? out - m : nullptr;
    a.lo = m;
    a.hi = m + n;
    a.offsets = nullptr;
    a.nstr = 0;
    a.shift = 0;
    a.flag = flag;
    a.results = nullptr;
    a.first = first;
    a.count = count;
    a.scalar_store = (op == kOpTo && (addr(out) & 15u) != (addr(in) & 15u)) ? 1 : 0;
    const LaunchShape sh = make_shape(get_params(op, 0, n), cus, n, m);
    if ((e = launch_main(op, false, sh, a, stream)) != hipSuccess)
        return hip_fail(e, "kernel launch");
    return UTF16WF_OK;
}

int check_u16(const void *p, const char *name) {
    if (addr(p) & 1u)
        return fail(UTF16WF_EALIGN, "%s is not 2-byte aligned", name);
    return UTF16WF_OK;
}

int batch_call(int op, const uint16_t *in, uint16_t *out, const int64_t *offsets, int64_t nstr,
               uint8_t *results, int64_t *first, int64_t *count, int64_t units_hint, hipStream_t stream) {
    int rc = check_op(op);
    if (rc != UTF16WF_OK)
        return rc;
    if (nstr < 0)
        return fail(UTF16WF_EINVAL, "num_strings < 0");
    if (units_hint < 0)
        return fail(UTF16WF_EINVAL, "units_hint < 0");
    if (nstr == 0)
        return UTF16WF_OK;
    if (!in || !offsets)
        return fail(UTF16WF_EINVAL, "null buffer or offsets");
    if (op == kOpTo && !out)
        return fail(UTF16WF_EINVAL, "null output");
    if (op == kOpToInplace && out && out != in)
        return fail(UTF16WF_EINVAL, "in-place call with a distinct output");
    if (op == kOpIs && !results)
        return fail(UTF16WF_EINVAL, "null results");
    if (op == kOpLocate && (!first || !count))
        return fail(UTF16WF_EINVAL, "null first_bad or count");
    if ((rc = check_u16(in, "in")) != UTF16WF_OK)
        return rc;
    if (out && (rc = check_u16(out, "out")) != UTF16WF_OK)
        return rc;
    if (addr(offsets) & 7u)
        return fail(UTF16WF_EALIGN, "offsets not 8-byte aligned");
    if (op == kOpLocate && ((addr(first) | addr(count)) & 7u))
        return fail(UTF16WF_EALIGN, "first_bad/count not 8-byte aligned");
    if (op == kOpTo && out == in)
        op = kOpToInplace;
    // The units a batch spans are on the device; with a size hint they are
    // known here: in[off[0], off[B]) and out[off[0], off[B]) overlap exactly
    // when the two pointers lie less than that span apart.
    if (op == kOpTo && units_hint > 0 && overlap_not_equal(in, out, units_hint))
        return fail(UTF16WF_EOVERLAP, "input and output lie %lld bytes apart, closer than the %lld units the batch spans",
                    (long long)(addr(in) > addr(out) ? addr(in) - addr(out) : addr(out) - addr(in)),
                    (long long)units_hint);

    int dev, cus;
    if ((rc = current_device(&dev)) != UTF16WF_OK)
        return rc;
    if ((rc = device_cus(dev, &cus)) != UTF16WF_OK)
        return rc;
    hipError_t e;
    // few long strings (or an unknown total): check each string's head first
    // so the main pass can skip strings whose first mismatch lies near their
    // start; the head check also sets every result's initial value
    const bool head = op == kOpIs && nstr <= 65536 && (units_hint == 0 || units_hint / nstr >= 8192);
    if (op == kOpIs && !head) {
        if ((e = launch_fill_u8(results, 1, nstr, stream)) != hipSuccess)
            return hip_fail(e, "fill results");
    } else if (op == kOpLocate) {
        if ((e = launch_fill_locate(first, count, nstr, stream)) != hipSuccess)
            return hip_fail(e, "fill first_bad and count");
    }
    const int64_t m = (int64_t)((addr(in) & 15u) >> 1);
    KernelArgs a{};
    a.in = in - m;
    uint16_t *dst = nullptr;
    if (op == kOpTo)
        dst = out;
    else if (op == kOpToInplace)
        dst = const_cast<uint16_t *>(in);
    a.out = dst ? dst - m : nullptr;
    a.lo = 0;
    a.hi = 0;
    a.offsets = offsets;
    a.nstr = nstr;
    a.shift = (int32_t)m;
    a.flag = nullptr;
    a.results = results;
    a.first = first;
    a.count = count;
    a.scalar_store = (op == kOpTo && (addr(out) & 15u) != (addr(in) & 15u)) ? 1 : 0;
    if (head) {
        if ((e = launch_head_check(a.in, offsets, nstr, m, results, stream)) != hipSuccess)
            return hip_fail(e, "head check launch");
    }
    // A locate over few strings behaves like the flat locate: the waves of
    // whole workgroups end on one string and add their totals with atomics
    // on it, so it takes the flat shape, tuned for one string (few, large
    // workgroups), which keeps those atomics few (one 2^28-unit string with
    // errors throughout: 160 us in the shape tuned for a million strings,
    // 108 us in the flat one).
    const bool flat_shape = op == kOpLocate && nstr <= kLocateFlatShapeMax;
    const utf16wf_params p = get_params(op, flat_shape ? 0 : 1, units_hint > 0 ? units_hint : (int64_t)1 << 40);
    const LaunchShape sh = make_shape(p, cus, units_hint, 0);
    if ((e = launch_main(op, true, sh, a, stream)) != hipSuccess)
        return hip_fail(e, "kernel launch");
    return UTF16WF_OK;
}

// A batch repair into a distinct buffer whose span (offsets[B] - offsets[0]
// units) is known: the two ranges it touches overlap exactly when the
// buffers lie less than the span apart.
int check_batch_overlap(const uint16_t *in, const uint16_t *out, int64_t span) {
    if (out && out != in && overlap_not_equal(in, out, span))
        return fail(UTF16WF_EOVERLAP, "input and output overlap over the %lld units the batch spans",
                    (long long)span);
    return UTF16WF_OK;
}

}  // namespace

namespace utf16wf {

int validation_flag_on_device(const int64_t *offsets, int64_t nstr, int64_t buf_units, hipStream_t s,
                              int32_t *flag, int64_t ends[2]) {
    hipError_t e;
    if ((e = launch_fill_i32(flag, 0, 1, s)) != hipSuccess)
        return hip_fail(e, "fill flag");
    if ((e = launch_validate(offsets, nstr, buf_units, flag, s)) != hipSuccess)
        return hip_fail(e, "validate launch");
    int32_t bad = 0;
    if ((e = hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&ends[0], offsets, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&ends[1], offsets + nstr, 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "copy flag and offsets' ends");
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "synchronize");
    if (bad)
        return fail(UTF16WF_EOFFSETS, "offsets are not non-decreasing within [0, %lld]", (long long)buf_units);
    return UTF16WF_OK;
}

int check_validate_batch_args(const uint16_t *in, const uint16_t *out, const int64_t *offsets, int64_t nstr,
                              int64_t buf_units) {
    if (nstr < 0 || buf_units < 0)
        return fail(UTF16WF_EINVAL, "negative size");
    if (!in || !offsets)
        return fail(UTF16WF_EINVAL, "null buffer or offsets");
    int rc;
    if ((rc = check_u16(in, "in")) != UTF16WF_OK || (out && (rc = check_u16(out, "out")) != UTF16WF_OK))
        return rc;
    if (addr(offsets) & 7u)
        return fail(UTF16WF_EALIGN, "offsets not 8-byte aligned");
    return UTF16WF_OK;
}

int validate_batch_with(const uint16_t *in, const uint16_t *out, const int64_t *offsets, int64_t nstr,
                        int64_t buf_units, hipStream_t s, int32_t *flag) {
    int64_t ends[2];
    int rc = validation_flag_on_device(offsets, nstr, buf_units, s, flag, ends);
    if (rc != UTF16WF_OK)
        return rc;
    return check_batch_overlap(in, out, ends[1] - ends[0]);
}

int set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}

int strings_call(int op, int n, const uint16_t *const *src, uint16_t *const *dst, const int64_t *len,
                 uint32_t *results, uint32_t stamp, hipStream_t stream) {
    if (op != kOpTo && op != kOpIs)
        return fail(UTF16WF_EINVAL, "strings: op must be the repair or the check");
    if (n < 0 || n > kMultiMax)
        return fail(UTF16WF_EINVAL, "strings: at most %d strings per launch", kMultiMax);
    if (n > 0 && (!src || !len || (op == kOpTo && !dst)))
        return fail(UTF16WF_EINVAL, "strings: null array");
    if (op == kOpIs && n > 0 && (!results || (addr(results) & 3u)))
        return fail(results ? UTF16WF_EALIGN : UTF16WF_EINVAL, "strings: results must be 4-byte aligned words");
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (len[i] < 0)
            return fail(UTF16WF_EINVAL, "strings: length %d < 0", i);
        if (len[i] == 0)
            continue;
        if (!src[i] || (op == kOpTo && !dst[i]))
            return fail(UTF16WF_EINVAL, "strings: null pointer for string %d", i);
        if ((addr(src[i]) & 1u) || (op == kOpTo && (addr(dst[i]) & 1u)))
            return fail(UTF16WF_EALIGN, "strings: string %d is not 2-byte aligned", i);
        if (op == kOpTo && overlap_not_equal(src[i], dst[i], len[i]))
            return fail(UTF16WF_EOVERLAP, "strings: input and output of string %d overlap", i);
        total += len[i];
    }
    if (total == 0)
        return UTF16WF_OK;
    int dev, cus, rc;
    if ((rc = current_device(&dev)) != UTF16WF_OK || (rc = device_cus(dev, &cus)) != UTF16WF_OK)
        return rc;
    // each string is a frame of its own, tiled like a flat call of the
    // batch's total size
    const utf16wf_params p = get_params(op, 0, total);
    const int64_t T = 512LL * p.rows;
    MultiArgs a{};
    int64_t tiles = 0;
    for (int i = 0; i < n; ++i) {
        MultiString &m = a.s[i];
        m.tile0 = tiles;
        if (len[i] == 0)
            continue;
        const int64_t ph = (int64_t)((addr(src[i]) & 15u) >> 1);
        m.in = src[i] - ph;
        m.out = op == kOpTo ? dst[i] - ph : nullptr;
        m.lo = ph;
        m.hi = ph + len[i];
        m.scalar_store = (op == kOpTo && (addr(dst[i]) & 15u) != (addr(src[i]) & 15u)) ? 1 : 0;
        tiles += (m.hi + T - 1) / T - m.lo / T;
    }
    a.ntiles = tiles;
    a.n = n;
    a.results = results;
    a.stamp = stamp;
    LaunchShape sh;
    sh.rows = p.rows;
    sh.wg_waves = p.wg_waves;
    sh.nontemporal = p.nontemporal;
    sh.store_lines = p.store_lines;
    const int64_t waves = std::min<int64_t>(tiles, (int64_t)p.grid_per_cu * cus * p.wg_waves);
    sh.grid = (int)std::max<int64_t>(1, (waves + p.wg_waves - 1) / p.wg_waves);
    hipError_t e;
    if ((e = launch_multi(op, sh, a, stream)) != hipSuccess)
        return hip_fail(e, "strings: kernel launch");
    return UTF16WF_OK;
}

}  // namespace utf16wf

namespace {

struct Plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

}  // namespace

extern "C" {

int utf16wf_abi_version(void) { return 2; }

const char *utf16wf_last_error(void) { return g_err.c_str(); }

int utf16wf_device_cus(void) {
    int dev, cus;
    if (current_device(&dev) != UTF16WF_OK || device_cus(dev, &cus) != UTF16WF_OK)
        return 0;
    return cus;
}

int utf16_is_well_formed(const uint16_t *in, int64_t n, int32_t *result, void *stream) {
    if (n < 0)
        return fail(UTF16WF_EINVAL, "n < 0");
    if (!result || (n > 0 && !in))
        return fail(UTF16WF_EINVAL, "null pointer");
    if (addr(result) & 3u)
        return fail(UTF16WF_EALIGN, "result not 4-byte aligned");
    if (n > 0 && check_u16(in, "in") != UTF16WF_OK)
        return UTF16WF_EALIGN;
    return flat_call(kOpIs, in, nullptr, n, result, nullptr, nullptr, (hipStream_t)stream);
}

int utf16_to_well_formed(const uint16_t *in, uint16_t *out, int64_t n, void *stream) {
    if (n < 0)
        return fail(UTF16WF_EINVAL, "n < 0");
    if (n == 0)
        return UTF16WF_OK;
    if (!in || !out)
        return fail(UTF16WF_EINVAL, "null pointer");
    int rc;
    if ((rc = check_u16(in, "in")) != UTF16WF_OK || (rc = check_u16(out, "out")) != UTF16WF_OK)
        return rc;
    if (overlap_not_equal(in, out, n))
        return fail(UTF16WF_EOVERLAP, "input and output overlap without being equal");
    const int op = (in == out) ? kOpToInplace : kOpTo;
    return flat_call(op, in, out, n, nullptr, nullptr, nullptr, (hipStream_t)stream);
}

int utf16_to_well_formed_inplace(uint16_t *buf, int64_t n, void *stream) {
    return utf16_to_well_formed(buf, buf, n, stream);
}

int utf16_locate_ill_formed(const uint16_t *in, int64_t n, int64_t *first_bad, int64_t *count, void *stream) {
    if (n < 0)
        return fail(UTF16WF_EINVAL, "n < 0");
    if (!first_bad || !count || (n > 0 && !in))
        return fail(UTF16WF_EINVAL, "null pointer");
    if ((addr(first_bad) | addr(count)) & 7u)
        return fail(UTF16WF_EALIGN, "first_bad/count not 8-byte aligned");
    if (n > 0 && check_u16(in, "in") != UTF16WF_OK)
        return UTF16WF_EALIGN;
    return flat_call(kOpLocate, in, nullptr, n, nullptr, first_bad, count, (hipStream_t)stream);
}

int utf16wf_batch(int op, const uint16_t *in, uint16_t *out, const int64_t *offsets, int64_t num_strings,
                  uint8_t *results, int64_t *first_bad, int64_t *count, int64_t units_hint, void *stream) {
    return batch_call(op, in, out, offsets, num_strings, results, first_bad, count, units_hint,
                      (hipStream_t)stream);
}

int utf16_is_well_formed_batch(const uint16_t *buf, const int64_t *offsets, int64_t num_strings, uint8_t *results,
                               void *stream) {
    return batch_call(kOpIs, buf, nullptr, offsets, num_strings, results, nullptr, nullptr, 0, (hipStream_t)stream);
}

int utf16_to_well_formed_batch(const uint16_t *in, uint16_t *out, const int64_t *offsets, int64_t num_strings,
                               void *stream) {
    return batch_call(kOpTo, in, out, offsets, num_strings, nullptr, nullptr, nullptr, 0, (hipStream_t)stream);
}

int utf16_to_well_formed_batch_inplace(uint16_t *buf, const int64_t *offsets, int64_t num_strings, void *stream) {
    return batch_call(kOpToInplace, buf, buf, offsets, num_strings, nullptr, nullptr, nullptr, 0,
                      (hipStream_t)stream);
}

int utf16_locate_ill_formed_batch(const uint16_t *buf, const int64_t *offsets, int64_t num_strings,
                                  int64_t *first_bad, int64_t *count, void *stream) {
    return batch_call(kOpLocate, buf, nullptr, offsets, num_strings, nullptr, first_bad, count, 0,
                      (hipStream_t)stream);
}

int utf16wf_validate_offsets(const int64_t *offsets, int64_t num_strings, int64_t buf_units, void *stream) {
    if (num_strings < 0 || buf_units < 0)
        return fail(UTF16WF_EINVAL, "negative size");
    if (!offsets)
        return fail(UTF16WF_EINVAL, "null offsets");
    if (addr(offsets) & 7u)
        return fail(UTF16WF_EALIGN, "offsets not 8-byte aligned");
    int dev, rc;
    Workspace *ws;
    if ((rc = current_device(&dev)) != UTF16WF_OK || (rc = workspace(dev, &ws)) != UTF16WF_OK)
        return rc;
    // the device flag is shared by every validation on this device; the call
    // is synchronous, so holding the lock for its duration serialises them
    std::lock_guard<std::mutex> lk(g_validate_mu[dev]);
    int64_t ends[2];
    return validation_flag_on_device(offsets, num_strings, buf_units, (hipStream_t)stream, ws->flag, ends);
}

int utf16wf_validate_batch(const uint16_t *in, const uint16_t *out, const int64_t *offsets, int64_t num_strings,
                           int64_t buf_units, void *stream) {
    int rc = check_validate_batch_args(in, out, offsets, num_strings, buf_units);
    if (rc != UTF16WF_OK)
        return rc;
    int dev;
    Workspace *ws;
    if ((rc = current_device(&dev)) != UTF16WF_OK || (rc = workspace(dev, &ws)) != UTF16WF_OK)
        return rc;
    std::lock_guard<std::mutex> lk(g_validate_mu[dev]);
    return validate_batch_with(in, out, offsets, num_strings, buf_units, (hipStream_t)stream, ws->flag);
}

int utf16wf_batch_plan_create(int op, const uint16_t *in, uint16_t *out, const int64_t *offsets,
                              int64_t num_strings, uint8_t *results, void *stream, void **plan) {
    if (!plan)
        return fail(UTF16WF_EINVAL, "null plan pointer");
    *plan = nullptr;
    int rc = check_op(op);
    if (rc != UTF16WF_OK)
        return rc;
    if (op == kOpLocate)
        return fail(UTF16WF_EINVAL, "plans support is / to / to_inplace");
    if (num_strings < 0)
        return fail(UTF16WF_EINVAL, "num_strings < 0");
    if (num_strings > 0) {
        // same checks the direct call makes, before any HIP call
        if (!in || !offsets || (op == kOpTo && !out) || (op == kOpIs && !results))
            return fail(UTF16WF_EINVAL, "null pointer");
        if ((rc = check_u16(in, "in")) != UTF16WF_OK || (out && (rc = check_u16(out, "out")) != UTF16WF_OK))
            return rc;
        if (addr(offsets) & 7u)
            return fail(UTF16WF_EALIGN, "offsets not 8-byte aligned");
    }
    Plan *p = new (std::nothrow) Plan;
    if (!p)
        return fail(UTF16WF_ENOMEM, "plan allocation");
    int dev;
    if ((rc = current_device(&dev)) != UTF16WF_OK) {
        delete p;
        return rc;
    }
    p->device = dev;
    // the units the offsets span now pick the captured launch's shape (as a
    // size hint does for a direct call); later contents stay correct
    int64_t units = 0;
    hipError_t e;
    if (num_strings > 0) {
        int64_t ends[2] = {0, 0};
        hipStream_t st = (hipStream_t)stream;
        if ((e = hipMemcpyAsync(&ends[0], offsets, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipMemcpyAsync(&ends[1], offsets + num_strings, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
            delete p;
            return hip_fail(e, "reading the offsets' ends");
        }
        units = std::max<int64_t>(0, ends[1] - ends[0]);
        if (op == kOpTo && (rc = check_batch_overlap(in, out, units)) != UTF16WF_OK) {
            delete p;
            return rc;
        }
    }
    hipStream_t cap;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        delete p;
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = batch_call(op, in, out, offsets, num_strings, results, nullptr, nullptr, units, cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (rc != UTF16WF_OK || e != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        delete p;
        return rc != UTF16WF_OK ? rc : hip_fail(e, "hipStreamEndCapture");
    }
    p->graph = g;
    e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete p;
        return hip_fail(e, "hipGraphInstantiate");
    }
    *plan = p;
    return UTF16WF_OK;
}

int utf16wf_batch_plan_launch(void *plan, void *stream) {
    if (!plan)
        return fail(UTF16WF_EINVAL, "null plan");
    Plan *p = static_cast<Plan *>(plan);
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "hipGraphLaunch");
    return UTF16WF_OK;
}

int utf16wf_batch_plan_destroy(void *plan) {
    if (!plan)
        return UTF16WF_OK;
    Plan *p = static_cast<Plan *>(plan);
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    delete p;
    return UTF16WF_OK;
}

int utf16wf_set_params(int op, int batch, int size_class_, const utf16wf_params *p) {
    if (check_op(op) != UTF16WF_OK)
        return UTF16WF_EINVAL;
    if (!p || (batch != 0 && batch != 1) || size_class_ < -1 || size_class_ >= kClasses)
        return fail(UTF16WF_EINVAL, "bad tuning key");
    if (!params_ok(*p))
        return fail(UTF16WF_EINVAL,
                    "bad parameters (rows %d, wg_waves %d, grid_per_cu %d, nontemporal %d, store_lines %d)", p->rows,
                    p->wg_waves, p->grid_per_cu, p->nontemporal, p->store_lines);
    std::lock_guard<std::mutex> lk(g_param_mu);
    init_params_locked();
    if (size_class_ < 0) {
        for (int c = 0; c < kClasses; ++c) {
            g_params[op][batch][c] = *p;
            g_params_set[op][batch][c] = true;
        }
    } else {
        g_params[op][batch][size_class_] = *p;
        g_params_set[op][batch][size_class_] = true;
    }
    return UTF16WF_OK;
}

int utf16wf_get_params(int op, int batch, int64_t n, utf16wf_params *p) {
    if (check_op(op) != UTF16WF_OK)
        return UTF16WF_EINVAL;
    if (!p || (batch != 0 && batch != 1) || n < 0)
        return fail(UTF16WF_EINVAL, "bad tuning key");
    *p = get_params(op, batch, n);
    return UTF16WF_OK;
}

int utf16wf_reset_params(void) {
    std::lock_guard<std::mutex> lk(g_param_mu);
    g_params_init = false;
    init_params_locked();
    return UTF16WF_OK;
}

int utf16_to_well_formed_host(const uint16_t *h_in, uint16_t *h_out, int64_t n, int64_t chunk_units) {
    if (n < 0 || chunk_units < 0)
        return fail(UTF16WF_EINVAL, "negative size");
    if (n == 0)
        return UTF16WF_OK;
    if (!h_in || !h_out)
        return fail(UTF16WF_EINVAL, "null pointer");
    int rc;
    if ((rc = check_u16(h_in, "h_in")) != UTF16WF_OK || (rc = check_u16(h_out, "h_out")) != UTF16WF_OK)
        return rc;
    if (overlap_not_equal(h_in, h_out, n))
        return fail(UTF16WF_EOVERLAP, "host input and output overlap without being equal");
    const int64_t chunk = std::min<int64_t>(n, chunk_units > 0 ? chunk_units : (int64_t)1 << 23);
    const int64_t nchunks = (n + chunk - 1) / chunk;
    const int stages = (int)std::min<int64_t>(kHostStages, nchunks);
    // input and output staging of every stage start 128-byte aligned
    const int64_t stride = (chunk + 2 + 63) / 64 * 64;
    const size_t need = (size_t)stages * 2 * (size_t)stride * sizeof(uint16_t);
    int dev;
    if ((rc = current_device(&dev)) != UTF16WF_OK)
        return rc;
    // Reuse the device's cached staging buffer, streams and events when they
    // are free and the staging is modest; otherwise (a concurrent call, or
    // very large chunks) use private ones for this call.
    HostStaging &cache = g_host_staging[dev];
    std::unique_lock<std::mutex> lk(cache.mu, std::try_to_lock);
    const bool cached = lk.owns_lock() && need <= kHostStagingCacheBytes;
    HostStaging priv;
    HostStaging &hs = cached ? cache : priv;
    hipError_t e;
    if (hs.bytes < need) {
        if (hs.buf)
            (void)hipFree(hs.buf);
        hs.buf = nullptr;
        hs.bytes = 0;
        if ((e = hipMalloc((void **)&hs.buf, need)) != hipSuccess)
            return hip_fail(e, "hipMalloc(staging)");
        hs.bytes = need;
    }
    rc = hs.ensure_streams();
    // Two streams, one per copy direction: copies in run back to back on
    // `in`, repairs and copies out on `out`; events hand each staging slot
    // from one to the other, so both PCIe directions stay busy.
    for (int64_t c = 0; c < nchunks && rc == UTF16WF_OK; ++c) {
        const int s = (int)(c % stages);
        uint16_t *d_in = hs.buf + (size_t)s * 2 * stride;
        uint16_t *d_out = d_in + stride;
        const int64_t a = c * chunk, b = std::min(n, a + chunk);
        const int64_t ca = a > 0 ? a - 1 : a, cb = b < n ? b + 1 : b;  // one unit of context each side
        if (c >= stages && (e = hipStreamWaitEvent(hs.in, hs.freed[s], 0)) != hipSuccess) {
            rc = hip_fail(e, "wait slot");
            break;
        }
        if ((e = hipMemcpyAsync(d_in, h_in + ca, (size_t)(cb - ca) * 2, hipMemcpyHostToDevice, hs.in)) !=
                hipSuccess ||
            (e = hipEventRecord(hs.loaded[s], hs.in)) != hipSuccess ||
            (e = hipStreamWaitEvent(hs.out, hs.loaded[s], 0)) != hipSuccess) {
            rc = hip_fail(e, "copy in");
            break;
        }
        if ((rc = utf16_to_well_formed(d_in, d_out, cb - ca, hs.out)) != UTF16WF_OK)
            break;
        if ((e = hipMemcpyAsync(h_out + a, d_out + (a - ca), (size_t)(b - a) * 2, hipMemcpyDeviceToHost,
                                hs.out)) != hipSuccess ||
            (e = hipEventRecord(hs.freed[s], hs.out)) != hipSuccess) {
            rc = hip_fail(e, "copy out");
            break;
        }
    }
    for (hipStream_t st : {hs.in, hs.out})
        if (st && (e = hipStreamSynchronize(st)) != hipSuccess && rc == UTF16WF_OK)
            rc = hip_fail(e, "synchronize");
    if (!cached)
        priv.release();
    return rc;
}

int utf16wf_copy_units(const uint16_t *in, uint16_t *out, int64_t n, void *stream) {
    if (n < 0)
        return fail(UTF16WF_EINVAL, "n < 0");
    if (n == 0)
        return UTF16WF_OK;
    if (!in || !out)
        return fail(UTF16WF_EINVAL, "null pointer");
    int rc;
    if ((rc = check_u16(in, "in")) != UTF16WF_OK || (rc = check_u16(out, "out")) != UTF16WF_OK)
        return rc;
    if ((addr(in) & 15u) != (addr(out) & 15u))
        return fail(UTF16WF_EALIGN, "copy needs equal alignment of in and out modulo 16");
    if (in == out || overlap_not_equal(in, out, n))
        return fail(UTF16WF_EOVERLAP, "copy buffers overlap");
    int dev, cus;
    if ((rc = current_device(&dev)) != UTF16WF_OK || (rc = device_cus(dev, &cus)) != UTF16WF_OK)
        return rc;
    const int64_t m = (int64_t)((addr(in) & 15u) >> 1);
    const LaunchShape sh = make_shape(get_params(kOpTo, 0, n), cus, n, m);
    hipError_t e = launch_copy(in - m, out - m, m, m + n, sh, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "copy launch");
    return UTF16WF_OK;
}

}  // extern "C"
