// UTF-16 well-formedness check and repair kernels for gfx950 (CDNA4).
//
// What is computed (arXiv 2601.06349): unit i is mismatched when it is a high
// surrogate whose successor is not a low surrogate, or a low surrogate whose
// predecessor is not a high surrogate; units outside the string count as
// non-surrogates (Sec. 1 definition; Sec. 3.1 block formulation and edge
// cases). Repair writes U+FFFD over mismatched units (Sec. 3.1 blend).
//
// How it maps to the GPU. The work is a stream over HBM with a few integer
// operations per unit, so the kernels are built for bandwidth, not for the
// matrix cores:
//   * A tile is R rows of 512 units handled by one wave; each lane issues one
//     16-byte load per row (8 units), so a row is 1 KiB of contiguous,
//     coalesced memory and a lane keeps R loads in flight.
//   * The paper loads every block twice at a one-unit offset to see each
//     unit's predecessor (Sec. 3.1, "lookback"). Here each unit is loaded
//     once: the 8 units of a lane are classified into per-byte flags with
//     SWAR on their high bytes (the top six bits decide the class, Sec. 3.3),
//     and the one flag a lane needs from each neighbour lane comes from a
//     wave ballot (one bit per lane), shifted by one lane on the scalar unit.
//     Across rows the carry is bit 63 / bit 0 of the neighbouring row's
//     ballot. Only at the two ends of a tile is a unit of context read from
//     memory, and only when it can matter (the first unit of the tile is a
//     low surrogate, or the last one is a high surrogate).
//   * The presence of any mismatch in a row is one more ballot (Sec. 3.1's
//     branchy fast path); rows without one store the loaded data unchanged,
//     and in place they store nothing (Sec. 3.2, in-place production
//     variant).
//   * No loop-carried state between tiles (Sec. 3.1 discussion), so waves
//     take contiguous runs of tiles and never communicate.
//   * Ragged batches: the repair marks string starts in a per-wave LDS
//     bitmap, filled from the offsets that fall inside the tile; a start cuts
//     the pairing between a unit and its predecessor. The check and the
//     locate keep all rows of a lane in one set of flag words (row r at bit
//     7 - r of each byte), compute the mismatches of the whole tile as if it
//     were one string, and let each lane of the tile's offsets take one
//     string: it tests its own range of units, and the pairs its two ends
//     cut (span_planes).
//   * Up to 32 separate strings, each at its own address (a serving batch),
//     run in one launch: each string is tiled alone, as a flat call's frame.
#include "kernels.h"

namespace utf16wf {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxWgWaves = 16;
constexpr int64_t kRowUnits = 512;  // 64 lanes x 8 units
constexpr uint32_t kRepl2 = 0xFFFDFFFDu;

// ------------------------------------------------------------- memory ops

template <bool NT>
__device__ __forceinline__ u32x4 ld16(const uint16_t *p) {
    const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
    if constexpr (NT)
        return __builtin_nontemporal_load(q);
    else
        return *q;
}

template <bool NT>
__device__ __forceinline__ void st16(uint16_t *p, u32x4 v) {
    u32x4 *q = reinterpret_cast<u32x4 *>(p);
    if constexpr (NT)
        __builtin_nontemporal_store(v, q);
    else
        *q = v;
}

__device__ __forceinline__ uint32_t unit_of(u32x4 v, int j) {
    uint32_t d = (j < 2) ? v.x : (j < 4) ? v.y : (j < 6) ? v.z : v.w;
    return (j & 1) ? (d >> 16) : (d & 0xFFFFu);
}

// Units u0..u0+7 with those outside [lo, hi) read as 0 (a non-surrogate);
// needs hi > lo. Every load reads a unit inside [lo, hi) (its index clamped
// there) and the select comes after, so the eight loads carry no branch and
// issue together under one wait.
__device__ __forceinline__ u32x4 ld_partial(const uint16_t *in, int64_t u0, int64_t lo, int64_t hi) {
    uint32_t w[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int64_t a = u0 + 2 * d, b = a + 1;
        const uint32_t x = in[min(max(a, lo), hi - 1)];
        const uint32_t y = in[min(max(b, lo), hi - 1)];
        w[d] = ((a >= lo && a < hi) ? x : 0u) | ((b >= lo && b < hi) ? y << 16 : 0u);
    }
    return (u32x4){w[0], w[1], w[2], w[3]};
}

// The same eight units, each load under its own bounds test. The batch
// kernel's edge tiles (the buffer's first and last) load this way: the
// clamped form above, or row tests on scalar registers, changed the register
// allocation and scheduling of the batch kernel's main loop and cost its
// interior tiles 5 to 20 % (measured on the 1,000,000-string, the
// 4096-string Zipf and the 1024-unit string batches).
__device__ __forceinline__ u32x4 ld_units(const uint16_t *in, int64_t u0, int64_t lo, int64_t hi) {
    uint32_t w[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int64_t a = u0 + 2 * d, b = a + 1;
        const uint32_t x = (a >= lo && a < hi) ? (uint32_t)in[a] : 0u;
        const uint32_t y = (b >= lo && b < hi) ? (uint32_t)in[b] : 0u;
        w[d] = x | (y << 16);
    }
    return (u32x4){w[0], w[1], w[2], w[3]};
}

// Store unit j of v to out[u0 + j] when u0 + j is in [lo, hi) and byte j of
// the 64-bit flag word `sel` has bit 7 set.
__device__ __forceinline__ void st_partial(uint16_t *out, int64_t u0, int64_t lo, int64_t hi, u32x4 v,
                                           uint64_t sel) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int64_t u = u0 + j;
        if (u >= lo && u < hi && ((sel >> (8 * j + 7)) & 1))
            out[u] = (uint16_t)unit_of(v, j);
    }
}

// One row of a tile that crosses lo or hi (hi > lo): the row starting at
// unit r0 (the same for the whole wave) is loaded with 16-byte vectors when
// it lies inside [lo, hi), not at all when it lies outside, and unit by unit
// only when it straddles an end. The tests are on wave-uniform values, so
// they are scalar branches. in + r0 is 16-byte aligned.
template <bool NT>
__device__ __forceinline__ u32x4 ld_row(const uint16_t *in, int64_t r0, int lane, int64_t lo, int64_t hi) {
    const int64_t u0 = r0 + (int64_t)lane * 8;
    if (r0 >= lo && r0 + kRowUnits <= hi)
        return ld16<NT>(in + u0);
    if (r0 + kRowUnits <= lo || r0 >= hi)
        return (u32x4){0u, 0u, 0u, 0u};
    return ld_partial(in, u0, lo, hi);
}

template <bool NT>
__device__ __forceinline__ void st_row(uint16_t *out, int64_t r0, int lane, int64_t lo, int64_t hi, u32x4 v) {
    const int64_t u0 = r0 + (int64_t)lane * 8;
    if (r0 >= lo && r0 + kRowUnits <= hi)
        st16<NT>(out + u0, v);
    else if (r0 + kRowUnits > lo && r0 < hi)
        st_partial(out, u0, lo, hi, v, 0x8080808080808080ull);
}

// ---------------------------------------------------------- classification
//
// Flags are kept one byte per unit: bit 7 of byte j of a 32-bit word is the
// flag of unit j (A = units 0..3 of a lane, B = units 4..7).

// Byte j of the result is the high byte of unit j of the dwords (lo, hi).
__device__ __forceinline__ uint32_t high_bytes(uint32_t lo_dw, uint32_t hi_dw) {
    return __builtin_amdgcn_perm(hi_dw, lo_dw, 0x07050301u);
}

// From four high bytes: h = 0xD8..0xDB (high surrogate), l = 0xDC..0xDF.
__device__ __forceinline__ void flags4(uint32_t hb, uint32_t &h, uint32_t &l) {
    // A byte of x is zero exactly when its unit is a surrogate. The low three
    // bits of every byte of x are zero, so the borrow of the zero-byte test
    // never produces a false flag.
    const uint32_t x = (hb & 0xF8F8F8F8u) ^ 0xD8D8D8D8u;
    const uint32_t s = (x - 0x01010101u) & ~x & 0x80808080u;
    l = s & (hb << 5);  // bit 2 of the high byte separates 0xDC.. from 0xD8..
    h = s ^ l;
}

// Four bits (bit j = unit j) to byte flags (bit 7 of byte j).
__device__ __forceinline__ uint32_t spread4(uint32_t b) {
    return ((b & 0xFu) * 0x00204081u & 0x01010101u) << 7;
}

// Mismatch flags of a lane's 8 units from their high / low flags (hA, lA:
// units 0..3; hB, lB: units 4..7), the string-start flags sA, sB (a start
// cuts the unit from its predecessor), whether the unit before the lane's
// first is a high that may pair (hp) and whether the unit after its last is
// a low that may pair (ln): a high whose successor is not a low, or a low
// whose predecessor is not a high.
__device__ __forceinline__ void mismatches(uint32_t hA, uint32_t hB, uint32_t lA, uint32_t lB, uint32_t sA,
                                           uint32_t sB, uint32_t hp, uint32_t ln, uint32_t &badA, uint32_t &badB) {
    const uint32_t lAp = lA & ~sA, lBp = lB & ~sB;
    const uint32_t psA = ((hA << 8) | (hp << 7)) & ~sA;  // predecessor is high
    const uint32_t psB = ((hB << 8) | (hA >> 24)) & ~sB;
    const uint32_t nsA = (lAp >> 8) | (lBp << 24);        // successor is low
    const uint32_t nsB = (lBp >> 8) | (ln << 31);
    badA = (hA & ~nsA) | (lA & ~psA);
    badB = (hB & ~nsB) | (lB & ~psB);
}

// Byte flags to 0xFF bytes.
__device__ __forceinline__ uint32_t byte_mask(uint32_t f) { return f | (f - (f >> 7)); }

// Replace flagged units of v with U+FFFD.
__device__ __forceinline__ u32x4 repair(u32x4 v, uint32_t badA, uint32_t badB) {
    const uint32_t mA = byte_mask(badA), mB = byte_mask(badB);
    const uint32_t m0 = __builtin_amdgcn_perm(mA, mA, 0x01010000u);
    const uint32_t m1 = __builtin_amdgcn_perm(mA, mA, 0x03030202u);
    const uint32_t m2 = __builtin_amdgcn_perm(mB, mB, 0x01010000u);
    const uint32_t m3 = __builtin_amdgcn_perm(mB, mB, 0x03030202u);
    u32x4 o;
    o.x = (v.x & ~m0) | (kRepl2 & m0);
    o.y = (v.y & ~m1) | (kRepl2 & m1);
    o.z = (v.z & ~m2) | (kRepl2 & m2);
    o.w = (v.w & ~m3) | (kRepl2 & m3);
    return o;
}

// 16 bytes starting `sh` bytes (even, 2..14) into the 32 bytes a|b.
__device__ __forceinline__ u32x4 realign(u32x4 a, u32x4 b, uint32_t sh) {
    const uint32_t k = sh & 3u;  // 0 or 2: byte shift inside a dword
    u32x4 o;
    switch (sh >> 2) {
    case 0:
        o = (u32x4){__builtin_amdgcn_alignbyte(a.y, a.x, k), __builtin_amdgcn_alignbyte(a.z, a.y, k),
                    __builtin_amdgcn_alignbyte(a.w, a.z, k), __builtin_amdgcn_alignbyte(b.x, a.w, k)};
        break;
    case 1:
        o = (u32x4){__builtin_amdgcn_alignbyte(a.z, a.y, k), __builtin_amdgcn_alignbyte(a.w, a.z, k),
                    __builtin_amdgcn_alignbyte(b.x, a.w, k), __builtin_amdgcn_alignbyte(b.y, b.x, k)};
        break;
    case 2:
        o = (u32x4){__builtin_amdgcn_alignbyte(a.w, a.z, k), __builtin_amdgcn_alignbyte(b.x, a.w, k),
                    __builtin_amdgcn_alignbyte(b.y, b.x, k), __builtin_amdgcn_alignbyte(b.z, b.y, k)};
        break;
    default:
        o = (u32x4){__builtin_amdgcn_alignbyte(b.x, a.w, k), __builtin_amdgcn_alignbyte(b.y, b.x, k),
                    __builtin_amdgcn_alignbyte(b.z, b.y, k), __builtin_amdgcn_alignbyte(b.w, b.z, k)};
        break;
    }
    return o;
}

// Output whose address phase differs from the input's by ks units (1..7):
// the 16-byte-aligned output vector a lane owns holds the last ks units of
// the group before its own and the first 8 - ks of its own, so every store
// is one aligned vector except the first 8 - ks units of a tile (`head`,
// lane 0 of its first row) and its last ks units (`tail`, lane 63 of its
// last row), which go unit by unit. o: the lane's repaired units
// [u0, u0 + 8); pv: those of the group before (the lane before, or for
// lane 0 the previous row's lane 63).
template <bool NT>
__device__ __forceinline__ void store_shifted(uint16_t *out, int64_t u0, int64_t lo, int64_t hi, u32x4 o, u32x4 pv,
                                              uint32_t ks, bool head, bool tail) {
    constexpr uint64_t kAll = 0x8080808080808080ull;
    const int64_t c0 = u0 - (int64_t)ks;  // the aligned vector: units [c0, c0 + 8)
    if (head) {
        st_partial(out, u0, lo, hi, o, kAll & ((1ull << (8 * (8 - ks))) - 1));
    } else {
        const u32x4 c = realign(pv, o, 16u - 2u * ks);
        if (c0 >= lo && c0 + 8 <= hi)
            st16<NT>(out + c0, c);
        else
            st_partial(out, c0, lo, hi, c, kAll);
    }
    if (tail)
        st_partial(out, u0, lo, hi, o, kAll & ~((1ull << (8 * (8 - ks))) - 1));
}

// The previous lane's vector (lane 0: `last`), and lane 63's, for
// store_shifted. All lanes of the wave call these together.
__device__ __forceinline__ u32x4 prev_lane(u32x4 o, u32x4 last, int lane) {
    const u32x4 p = (u32x4){(uint32_t)__shfl_up((int)o.x, 1), (uint32_t)__shfl_up((int)o.y, 1),
                            (uint32_t)__shfl_up((int)o.z, 1), (uint32_t)__shfl_up((int)o.w, 1)};
    return lane == 0 ? last : p;
}
__device__ __forceinline__ u32x4 lane63(u32x4 o) {
    return (u32x4){(uint32_t)__builtin_amdgcn_readlane((int)o.x, 63), (uint32_t)__builtin_amdgcn_readlane((int)o.y, 63),
                   (uint32_t)__builtin_amdgcn_readlane((int)o.z, 63), (uint32_t)__builtin_amdgcn_readlane((int)o.w, 63)};
}

__device__ __forceinline__ bool is_high_unit(uint32_t u) { return (u & 0xFC00u) == 0xD800u; }
__device__ __forceinline__ bool is_low_unit(uint32_t u) { return (u & 0xFC00u) == 0xDC00u; }

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------ offsets

// The value of v in lane l (the same in every lane), read into scalar
// registers.
__device__ __forceinline__ int64_t lane_value(int64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// First index i in [a, b) with off[i] >= target, else b (off sorted). All
// lanes of the wave call it with the same arguments; probes 64 positions per
// round.
__device__ int64_t lower_bound_wave(const int64_t *off, int64_t a, int64_t b, int64_t target, int lane) {
    while (b - a > 64) {
        const int64_t step = (b - a + 63) >> 6;
        const int64_t idx = a + (int64_t)lane * step;
        const bool lt = idx < b && off[idx] < target;
        const int c = __popcll(__ballot(lt));
        if (c == 0)
            return a;
        const int64_t na = a + (int64_t)(c - 1) * step + 1;
        const int64_t nb = min(b, a + (int64_t)c * step);
        a = na;
        b = nb;
    }
    const int64_t idx = a + lane;
    const bool lt = idx < b && off[idx] < target;
    return a + __popcll(__ballot(lt));
}

struct TileStarts {
    int64_t kc;     // string holding unit tl (-1 if tl is before the first string)
    int64_t knext;  // first k with off[k] + shift >= th
    int64_t k0;     // first k with off[k] + shift >= tl (the scan's cursor)
    int64_t onext;  // off[knext] + shift (INT64_MAX past the last offset)
    bool next;      // a string starts at unit th
    bool inner;     // a string starts in (tl, th)
    bool any;       // a string starts in [tl, th) (the bitmap has a bit set)
    bool at_tl = false;  // a string starts at unit tl
};

// Marks the string starts in [tl, th) in the wave's bitmap (bit u - tl).
// `cursor` is the first k with off[k] + shift >= tl. The bitmap is cleared
// only when the previous tile left bits in it (`dirty`), so tiles inside one
// long string touch no LDS at all.
template <int R, bool BITMAP = true>
__device__ __forceinline__ TileStarts scan_starts(const int64_t *off, int64_t nstr, int64_t shift,
                                                  int64_t cursor, int64_t tl, int64_t th, uint32_t *bm,
                                                  int lane, bool &dirty, int64_t *o_first = nullptr) {
    constexpr int kWords = 16 * R;
    if (BITMAP && dirty) {
#pragma unroll
        for (int i = 0; i < (kWords + 63) / 64; ++i) {
            const int w = i * 64 + lane;
            if (w < kWords)
                bm[w] = 0u;
        }
        wave_lds_sync();
        dirty = false;
    }
    int64_t k = cursor, le = 0;
    bool next = false, inner = false, first_round = true;
    int64_t onext = INT64_MAX;
    for (;;) {
        const int64_t idx = k + lane;
        const int64_t o = idx <= nstr ? off[idx] + shift : INT64_MAX;
        if (first_round && o_first)
            *o_first = o;
        const bool lt = o < th;
        if (BITMAP && lt) {
            // with valid offsets tl <= o < th always holds here; the test
            // keeps malformed offsets from writing outside the bitmap
            const int64_t rel = o - tl;
            if (rel >= 0 && rel < 32 * kWords)
                atomicOr(&bm[rel >> 5], 1u << (rel & 31));
        }
        le += __popcll(__ballot(o <= tl));
        next = next || (__ballot(o == th) != 0);
        inner = inner || (__ballot(o > tl && lt) != 0);
        const int c = __popcll(__ballot(lt));
        k += c;
        if (c == 64) {
            // 64 equal offsets: a run of empty strings, which may go on for
            // millions; skip the rest of it with a search rather than reading
            // it 64 at a time (its start bit is set, and a run at tl counts
            // whole towards le)
            const int64_t o0 = lane_value(o, 0), o63 = lane_value(o, 63);
            if (o0 == o63) {
                const int64_t kend = lower_bound_wave(off, k, nstr + 1, o0 - shift + 1, lane);
                if (o0 <= tl)
                    le += kend - k;
                k = kend;
            }
        }
        if (c < 64) {
            onext = (int64_t)__shfl((long long)o, c);  // the first offset at or past th
            break;
        }
        first_round = false;
    }
    const bool any = BITMAP && k != cursor;
    if (any) {
        wave_lds_sync();
        dirty = true;
    }
    TileStarts ts{cursor + le - 1, k, cursor, onext, next, inner, any};
    ts.at_tl = le > 0;
    return ts;
}

// Bits of the 64-bit group mask m (row r of a tile: group 64 r + lane) that
// lie in groups [g0, g1].
__device__ __forceinline__ uint64_t groups_in(uint64_t m, int r, int g0, int g1) {
    const int lo = max(g0 - 64 * r, 0), hi = min(g1 - 64 * r, 63);
    if (lo > hi)
        return 0ull;
    const uint64_t upto = hi == 63 ? ~0ull : ((2ull << hi) - 1ull);
    return m & upto & ~((1ull << lo) - 1ull);
}

// Batch check and locate of a tile that holds string starts. The tile's
// mismatches and pairs were computed as in one string (a pair across a string
// start counts as a pair) for all rows at once: w4[lane] holds the lane's
// mismatch flags (x: units 0..3, y: units 4..7) and pair flags (z, w: the
// unit is a low after a high), unit j of row r at bit 8 (j & 3) + 7 - r;
// M[r] has bit `lane` set where the lane's row-r units hold a mismatch. Each
// lane takes one string: lane j of a round of 64 offsets (offsets kb + j)
// takes string kb + j - 1, whose units in the tile are [max(a, tl), min(o,
// th)) with a = offsets[kb + j - 1] and o = offsets[kb + j] (plus shift). Its
// mismatches are the ones in that range, plus a pair cut by its start (the
// unit at a is a low after a high) or by its end (the unit at o is) when that
// boundary lies inside the tile; boundaries at tl and th were cut when the
// tile was computed. The check clears the string's result; the locate adds
// its count and offers its first mismatch. o_first: offsets[cursor + lane]
// + shift (INT64_MAX past the last), cursor the first k with offsets[k] +
// shift >= tl. start_prev: where string cursor - 1 starts, if known
// (INT64_MIN otherwise; the locate then reads it). pre: the check with at
// most 4 rows, 64 R bytes of the wave's LDS; a string whose first and last
// groups are clean and that has groups between tests them with two reads of
// pre[g], the number of groups before g that hold a mismatch, filled when a
// string first needs it (otherwise, and for the locate, the middle groups'
// masks are tested row by row). Returns the start of the string holding unit
// th - 1, if known. All lanes of the wave call it together.
template <int OP, int R>
__device__ __forceinline__ int64_t span_planes(const KernelArgs &a, const int64_t *off, int64_t shift,
                                               int64_t cursor, int64_t o_first, int64_t tl, int64_t th, int lane,
                                               const uint4 *w4, const uint64_t (&M)[R], int64_t start_prev,
                                               uint8_t *pre) {
    constexpr int T = kRowUnits * R;
    constexpr uint64_t kUnits = 0x0101010101010101ull;  // bit 8 j: unit j of row 7
    int64_t kb = cursor, o = o_first;
    int32_t ac = -1;               // start of string kb - 1 relative to tl (-1: before the tile)
    int64_t ac_abs = start_prev;   // ... and absolute, if known
    bool pre_done = false;         // check: pre[] filled for this tile
    for (;;) {
        const int32_t orl = (int32_t)min(max(o - tl, (int64_t)-1), (int64_t)T + 1);
        int32_t arl = __shfl_up(orl, 1);
        if (lane == 0)
            arl = ac;
        const int64_t k = kb + lane - 1;
        const int64_t o63 = lane_value(o, 63);
        bool bad = false, need = false;  // check: a mismatch found / the middle groups still to test
        int g0n = 0, g1n = 0;
        if (k >= 0 && k < a.nstr && orl > 0 && arl < T && arl < orl) {
            const int ul = max(arl, 0), uh = min(orl, T);
            const int g0 = ul >> 3, g1 = (uh - 1) >> 3;
            const uint4 W0 = w4[g0 & 63], W1 = w4[g1 & 63];
            const uint64_t from0 = ~0ull << (8 * (ul & 7));        // units >= ul in its group
            const uint64_t upto1 = ~0ull >> (56 - 8 * ((uh - 1) & 7));  // units < uh in its group
            const uint64_t row0 = kUnits << (7 - (g0 >> 6)), row1 = kUnits << (7 - (g1 >> 6));
            const uint64_t bad0 = ((uint64_t)W0.y << 32 | W0.x) & row0 & from0;
            const uint64_t f0 = g0 == g1 ? bad0 & upto1 : bad0;
            const uint64_t f1 = g0 == g1 ? 0ull : ((uint64_t)W1.y << 32 | W1.x) & row1 & upto1;
            const uint64_t p0 = (uint64_t)W0.w << 32 | W0.z;
            const bool cs = arl > 0 && ((p0 >> (8 * (ul & 7) + 7 - (g0 >> 6))) & 1ull);
            bool ce = false;
            if (orl < T) {
                const int ge = uh >> 3;
                const uint4 We = w4[ge & 63];
                ce = ((((uint64_t)We.w << 32 | We.z) >> (8 * (uh & 7) + 7 - (ge >> 6))) & 1ull) != 0ull;
            }
            if constexpr (OP == kOpIs) {
                bad = cs || ce || f0 || f1;
                if constexpr (R <= 4) {
                    need = !bad && g1 - g0 >= 2;
                    g0n = g0;
                    g1n = g1;
                } else if (!bad && g1 - g0 >= 2) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        bad = bad || groups_in(M[r], r, g0 + 1, g1 - 1) != 0ull;
                }
            } else {
                constexpr int kNone = 0x7FFFFFFF;
                uint32_t cnt = (uint32_t)__popcll(f0) + (uint32_t)cs + (uint32_t)ce;
                int first = cs ? ul : f0 ? g0 * 8 + (__builtin_ctzll(f0) >> 3) : kNone;
                if (g1 - g0 >= 2) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        uint64_t m = groups_in(M[r], r, g0 + 1, g1 - 1);
                        while (m) {
                            const int l = __builtin_ctzll(m);
                            m &= m - 1ull;
                            const uint4 W = w4[l];
                            const uint64_t b = ((uint64_t)W.y << 32 | W.x) & (kUnits << (7 - r));
                            cnt += (uint32_t)__popcll(b);
                            if (first == kNone)
                                first = (64 * r + l) * 8 + (__builtin_ctzll(b) >> 3);
                        }
                    }
                }
                cnt += (uint32_t)__popcll(f1);
                if (first == kNone && f1)
                    first = g1 * 8 + (__builtin_ctzll(f1) >> 3);
                if (first == kNone && ce)
                    first = uh - 1;
                if (cnt) {
                    const int64_t start = arl >= 0 ? tl + arl : ac_abs != INT64_MIN ? ac_abs : off[k] + shift;
                    const uint64_t rel = (uint64_t)(tl + first - start);
                    // atomics even for a string wholly inside the tile: no
                    // slower than plain stores here, and where one wave saw
                    // whole strings tile after tile (1024-unit strings), plain
                    // 8-byte stores from many waves into shared lines took
                    // the locate from 140 to 151 us
                    atomicMin(reinterpret_cast<unsigned long long *>(a.first + k), (unsigned long long)rel);
                    atomicAdd(reinterpret_cast<unsigned long long *>(a.count + k), (unsigned long long)cnt);
                }
            }
        }
        if constexpr (OP == kOpIs) {
            if (__ballot(need)) {
                // strings whose first and last groups are clean and that have
                // groups between: pre[g] counts the mismatch groups before g
                // (g = 64 r + lane), filled once per tile when first needed
                if (!pre_done) {
                    uint32_t base = 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(M[r] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)M[r], 0u));
                        pre[r * 64 + lane] = (uint8_t)(base + below);  // at most 255: R <= 4
                        base += (uint32_t)__popcll(M[r]);
                    }
                    wave_lds_sync();
                    pre_done = true;
                }
                if (need)
                    bad = pre[g1n] != pre[g0n + 1];
            }
            if (bad)
                __hip_atomic_store(a.results + k, (uint8_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (o63 >= th) {
            const int c = __popcll(__ballot(o < th));
            return c > 0 ? lane_value(o, c - 1) : ac >= 0 ? tl + ac : ac_abs;
        }
        ac = __builtin_amdgcn_readlane(orl, 63);
        ac_abs = o63;
        kb += 64;
        const int64_t o0 = lane_value(o, 0);
        if (o0 == o63)  // 64 equal offsets: skip the rest of the run of empty strings
            kb = lower_bound_wave(off, kb, a.nstr + 1, o0 - shift + 1, lane);
        const int64_t idx = kb + lane;
        o = idx <= a.nstr ? off[idx] + shift : INT64_MAX;
    }
}

// ------------------------------------------------------------- the kernel

// OP: the operation; BATCH: ragged batch (else one buffer); R: rows per tile;
// NT: non-temporal loads and stores. SS, out-of-place repair: the output's
// address phase differs from the input's (stores are realigned); in-place
// repair: sector stores (only the 16-byte vectors that changed are written,
// instead of every 128-byte line that holds a change).
template <int OP, bool BATCH, int R, bool NT, bool SS>
__global__ void __launch_bounds__(1024) wf_kernel(KernelArgs a) {
    constexpr int64_t T = kRowUnits * R;
    constexpr int kWords = 16 * R;
    constexpr bool kFlatLocate = (OP == kOpLocate && !BATCH);
    // check and locate keep no start bitmap; their tiles with several strings
    // leave mismatch and pair bits here for span_strings
    constexpr bool kSpans = BATCH && (OP == kOpIs || OP == kOpLocate);
    __shared__ uint32_t s_bm[(BATCH && !kSpans) ? kMaxWgWaves * kWords : 1];
    __shared__ uint4 s_w4[kSpans ? kMaxWgWaves * 64 : 1];
    // the check with at most 4 rows: counts of mismatch groups before each
    // group, for span_planes (with 8 rows, measured slower on the 1024-unit
    // string batch than testing the middle groups' masks)
    constexpr bool kPre = kSpans && OP == kOpIs && R <= 4;
    __shared__ uint8_t s_pre[kPre ? kMaxWgWaves * 64 * R : 1];
    // OP_LOCATE: per-workgroup totals, published by the last wave (batch:
    // for the one string s_loc_k that the first reporting wave names)
    __shared__ unsigned long long s_loc_first, s_loc_k, s_loc_total;
    __shared__ uint32_t s_loc_count, s_loc_done;
    // (batch: only with few strings, whose tiles span many workgroups; with
    // many short ones each wave's last string is its own)
    const bool loc_wg = kFlatLocate || (OP == kOpLocate && BATCH && a.nstr <= 65536);
    if (loc_wg) {
        if (threadIdx.x == 0) {
            s_loc_first = ~0ull;
            s_loc_k = ~0ull;
            s_loc_total = 0ull;
            s_loc_count = 0u;
            s_loc_done = 0u;
        }
        __syncthreads();
    }

    const int lane = __lane_id();
    // the wave's slot in its workgroup. One buffer: known to the compiler as
    // wave-uniform, so tile indices, loop bounds and the edge tiles' row
    // tests live in scalar registers and an edge tile's rows load together.
    // Batch: left as is (see ld_units).
    const int wslot = BATCH ? (int)(threadIdx.x >> 6) : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wg_waves = blockDim.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * wg_waves;
    const int64_t wave = (int64_t)blockIdx.x * wg_waves + wslot;

    const uint16_t *in = a.in;
    uint16_t *out = a.out;
    const int64_t *off = a.offsets;
    const int64_t shift = a.shift;
    int64_t lo = a.lo, hi = a.hi;
    if constexpr (BATCH) {
        lo = off[0] + shift;
        hi = off[a.nstr] + shift;
    }
    if (hi <= lo)
        return;
    const int64_t t0 = lo / T, t1 = (hi + T - 1) / T;
    const int64_t per = (t1 - t0 + nwaves - 1) / nwaves;
    const int64_t tb = t0 + wave * per;
    const int64_t te = min(tb + per, t1);
    if (tb >= te && !loc_wg)
        return;  // (such locate waves without tiles still report to their workgroup)

    uint32_t *bm = (BATCH && !kSpans) ? s_bm + wslot * kWords : nullptr;
    uint4 *w4 = kSpans ? s_w4 + wslot * 64 : nullptr;
    uint8_t *pre = kPre ? s_pre + wslot * 64 * R : nullptr;
    int64_t o_first = 0;                     // span_strings: the tile's first 64 offsets
    int64_t span_k = -1, span_start = INT64_MIN;  // start of string span_k, if known
    bool bm_dirty = true;  // LDS starts with arbitrary contents
    // batch isWellFormed: string whose last tile this wave read was whole
    // inside it and clean (-1 if none)
    int64_t clean_k = -1;
    // batch: first string index of the wave's first tile. With many strings
    // the search is long and its result gates the tile's offsets scan, so it
    // runs first and the scan's loads then overlap the data loads; with few
    // (long) strings it is short and runs after the first tile's loads are
    // in flight (isWellFormed of few strings needs it before any load, for
    // its skip test). Measured on the 1M-string and 4096-string batches.
    int64_t cursor = -1;
    if constexpr (BATCH) {
        if (a.nstr > 65536)
            cursor = lower_bound_wave(off, 0, a.nstr + 1, tb * T - shift, lane);
    }

    // OP_LOCATE accumulators: count per lane, first index per wave. Flat:
    // the whole run; batch: consecutive tiles that lie inside one string
    // (loc_k), flushed with one pair of atomics when the string changes.
    uint64_t loc_first = ~0ull;
    uint32_t loc_count = 0;
    int64_t loc_k = -1;
    auto loc_flush = [&]() {
        uint32_t c = loc_count;
#pragma unroll
        for (int sh = 32; sh >= 1; sh >>= 1)
            c += __shfl_xor(c, sh);
        if (lane == 0 && c != 0) {
            atomicAdd(reinterpret_cast<unsigned long long *>(a.count + loc_k), (unsigned long long)c);
            atomicMin(reinterpret_cast<unsigned long long *>(a.first + loc_k), (unsigned long long)loc_first);
        }
        loc_count = 0;
        loc_first = ~0ull;
    };

    // batch isWellFormed of few strings: the first offset past the previous
    // tile (`nxt`, string `cursor` starts there) and the result byte of
    // string cursor - 1, read with the previous tile's loads (`known`: the
    // coming tile lies inside that string and pk holds its result)
    int64_t nxt = -1;
    uint8_t pk = 1;
    bool pk_valid = false;

    // flat OP_IS early exit: the result word drops to 0 once any wave has
    // seen a mismatch. The first poll waits (a wave that starts late skips
    // all its loads); later polls are issued with a tile's loads and read at
    // the next tile, so they add no latency.
    int32_t poll = 1;
    if constexpr (OP == kOpIs && !BATCH) {
        if (__hip_atomic_load(a.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
            return;
    }

    // output phase differing from the input's (SS): by ks units
    const uint32_t ks = SS ? (uint32_t)((reinterpret_cast<uintptr_t>(out) & 15u) >> 1) : 0u;
    u32x4 last = (u32x4){0u, 0u, 0u, 0u};  // SS: lane 63's repaired units of the previous row

    for (int64_t t = tb; t < te; ++t) {
        const int64_t tl = t * T, th = tl + T;
        if constexpr (OP == kOpIs && !BATCH) {
            if (poll == 0)
                return;
        }
        const bool interior = tl >= lo && th <= hi;
        u32x4 v[R];
        TileStarts ts{0, 0, 0, 0, false, false, false};

        // Batch isWellFormed of few (long) strings checks first whether the
        // whole tile lies in a string already known to be ill-formed; then
        // its data need not be read at all. With many short strings a tile
        // holds dozens of them, the check never fires, and the tile's loads
        // go first as for the other operations.
        const bool skip_first = BATCH && OP == kOpIs && a.nstr <= 65536;
        if (skip_first) {
            const bool known = pk_valid && nxt >= th;
            pk_valid = false;
            if (known) {
                // No offset falls in [tl, th): the tile lies inside string
                // cursor - 1, whose result came with the previous tile's
                // loads, so neither a scan nor a wait precedes this tile's
                // loads. Known ill-formed: jump to where the string ends.
                if (pk == 0) {
                    const int64_t tn = nxt / T;
                    if (tn > t + 1)
                        t = tn - 1;
                    continue;
                }
                ts = TileStarts{cursor - 1, cursor, cursor, nxt, nxt == th, false, false};
            } else {
                if (cursor < 0)
                    cursor = lower_bound_wave(off, 0, a.nstr + 1, tl - shift, lane);
                ts = scan_starts<R, !kSpans>(off, a.nstr, shift, cursor, tl, th, bm, lane, bm_dirty, &o_first);
                cursor = ts.knext;
                nxt = ts.onext;
                if (!ts.inner && ts.kc >= 0 && ts.kc < a.nstr &&
                    __hip_atomic_load(a.results + ts.kc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                    // jump to the tile where string kc ends: the tiles before
                    // it lie inside kc and need neither a scan nor a load
                    const int64_t tn = (off[ts.kc + 1] + shift) / T;
                    if (tn > t + 1) {
                        t = tn - 1;
                        cursor = ts.kc + 1;  // off[kc] < tn * T <= off[kc + 1]
                    }
                    continue;
                }
            }
        }
        if constexpr (BATCH) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t u0 = tl + ((int64_t)r * 64 + lane) * 8;
                v[r] = interior ? ld16<NT>(in + u0) : ld_units(in, u0, lo, hi);
            }
        } else if (interior) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[r] = ld16<NT>(in + tl + ((int64_t)r * 64 + lane) * 8);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[r] = ld_row<NT>(in, tl + (int64_t)r * kRowUnits, lane, lo, hi);
        }
        if constexpr (OP == kOpIs && !BATCH)
            poll = __hip_atomic_load(a.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (skip_first && nxt >= th + T && cursor >= 1 && cursor - 1 < a.nstr) {
            // the coming tile lies inside string cursor - 1: fetch its result
            // now, with this tile's loads
            pk = __hip_atomic_load(a.results + cursor - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            pk_valid = true;
        }
        if (BATCH && !skip_first) {
            if (cursor < 0)
                cursor = lower_bound_wave(off, 0, a.nstr + 1, tl - shift, lane);
            ts = scan_starts<R, !kSpans>(off, a.nstr, shift, cursor, tl, th, bm, lane, bm_dirty, &o_first);
            cursor = ts.knext;
        }
        // batch locate: does the whole tile lie inside one string?
        const bool single = BATCH && !ts.inner && ts.kc >= 0 && ts.kc < a.nstr;
        if constexpr (OP == kOpLocate && BATCH) {
            if (single && ts.kc != loc_k) {
                if (loc_k >= 0)
                    loc_flush();
                loc_k = ts.kc;
            }
        }

        if constexpr (kSpans) {
            // Check and locate: every row's flags in one set of words, row r
            // at bit 7 - r of each byte (the classification puts a flag at
            // bit 7), so the mismatches and pairs of all rows come from one
            // pass of the same arithmetic. Computed as in one string; string
            // starts inside the tile are handled by span_planes.
            uint32_t HA = 0, HB = 0, LA = 0, LB = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                uint32_t hA, lA, hB, lB;
                flags4(high_bytes(v[r].x, v[r].y), hA, lA);
                flags4(high_bytes(v[r].z, v[r].w), hB, lB);
                HA |= hA >> r;
                LA |= lA >> r;
                HB |= hB >> r;
                LB |= lB >> r;
            }
            // Neighbours of all rows at once: the previous lane's unit-7 high
            // flags and the next lane's unit-0 low flags (DPP wave shifts by
            // one lane). Lane 0 takes lane 63's flags one row up, lane 63
            // lane 0's one row down; the tile's ends take a unit of context,
            // cut by a string start at tl or th.
            const uint32_t h7 = HB >> 24, l0 = LA & 0xFFu;  // bits 7 - r of byte 0
            const uint32_t h7_63 = __builtin_amdgcn_readlane(h7, 63), l0_0 = __builtin_amdgcn_readlane(l0, 0);
            uint32_t cin = 0, cnx = 0;
            if ((l0_0 & 0x80u) && tl - 1 >= lo && !ts.at_tl)
                cin = is_high_unit(in[tl - 1]) ? 0x80u : 0u;
            if ((h7_63 & (0x80u >> (R - 1))) && th < hi && !ts.next)
                cnx = is_low_unit(in[th]) ? (0x80u >> (R - 1)) : 0u;
            uint32_t hp = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)h7, 0x138, 0xF, 0xF, true);  // wave_shr:1
            uint32_t ln = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)l0, 0x130, 0xF, 0xF, true);  // wave_shl:1
            if (lane == 0)
                hp = ((h7_63 >> 1) & (0xFFu << (8 - R))) | cin;
            if (lane == 63)
                ln = ((l0_0 << 1) & 0xFFu) | cnx;
            const uint32_t psA = (HA << 8) | hp, psB = (HB << 8) | (HA >> 24);  // predecessor is high
            const uint32_t nsA = (LA >> 8) | (LB << 24), nsB = (LB >> 8) | (ln << 24);  // successor is low
            const uint32_t badA = (HA & ~nsA) | (LA & ~psA), badB = (HB & ~nsB) | (LB & ~psB);
            const uint32_t anyb = badA | badB;
            if (single) {
                const uint64_t wb = __ballot(anyb != 0u);
                if constexpr (OP == kOpIs) {
                    // The whole tile is string kc: one store settles it. The
                    // clearing is published device-wide, for the skip test
                    // of the string's tiles not yet read, only when this wave
                    // found the string's previous tile clean: its errors are
                    // then sparse and few waves publish. Where they are dense
                    // every wave covering the string finds one in its first
                    // tile, and their coherent stores would queue (200 long
                    // strings with dense errors past their heads: 128 us when
                    // every finder published, 78 us under this rule; one
                    // error late in each: 270 us when none published, 208 us
                    // under it). Other clearings go through this XCD's
                    // cache, which the kernel's end writes back.
                    if (wb && lane == 0) {
                        if (skip_first && clean_k == ts.kc) {
                            if (__hip_atomic_load(a.results + ts.kc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                                __hip_atomic_store(a.results + ts.kc, (uint8_t)0, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        } else {
                            __hip_atomic_store(a.results + ts.kc, (uint8_t)0, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                    clean_k = wb ? -1 : ts.kc;
                } else if (wb) {
                    loc_count += (uint32_t)(__popc(badA) + __popc(badB));
                    if (loc_first == ~0ull) {
                        int r0 = 0;
                        uint64_t m0 = 0;
#pragma unroll
                        for (int r = R - 1; r >= 0; --r) {
                            const uint64_t m = __ballot(anyb & (0x80808080u >> r));
                            if (m) {
                                r0 = r;
                                m0 = m;
                            }
                        }
                        const int fl = __builtin_ctzll(m0);
                        const uint64_t fb = ((uint64_t)(uint32_t)__shfl((int)badB, fl) << 32) |
                                            (uint32_t)__shfl((int)badA, fl);
                        const int jf = __builtin_ctzll(fb & (0x0101010101010101ull << (7 - r0))) >> 3;
                        loc_first = (uint64_t)(tl + ((int64_t)r0 * 64 + fl) * 8 + jf - (off[loc_k] + shift));
                    }
                }
            } else {
                if constexpr (OP == kOpIs)
                    clean_k = -1;
                const uint32_t prA = LA & psA, prB = LB & psB;
                uint64_t M[R];
                uint64_t any = 0ull;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    M[r] = __ballot(anyb & (0x80808080u >> r));
                    any |= M[r];
                }
                any |= __ballot((prA | prB) != 0u);
                const int64_t sp = (span_k >= 0 && span_k == ts.k0 - 1) ? span_start : INT64_MIN;
                if (any) {
                    w4[lane] = (uint4){badA, badB, prA, prB};
                    wave_lds_sync();
                    span_start = span_planes<OP, R>(a, off, shift, ts.k0, o_first, tl, th, lane, w4, M, sp, pre);
                } else {
                    span_start = INT64_MIN;
                }
                span_k = ts.knext - 1;
            }
            continue;
        }

        // Phase 1: classify every row and ballot the two flags that
        // neighbouring lanes need: "my unit 7 is high" and "my unit 0 is a
        // low that may pair backwards" (not a string start). (Keeping the
        // flags live into phase 2 costs occupancy in the batch kernel but
        // measured faster than classifying again there.)
        uint32_t hA_[R], hB_[R], lA_[R], lB_[R], sbits[R];
        uint64_t hl[R], lf[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            flags4(high_bytes(v[r].x, v[r].y), hA_[r], lA_[r]);
            flags4(high_bytes(v[r].z, v[r].w), hB_[r], lB_[r]);
            sbits[r] = (BATCH && ts.any) ? (uint32_t)reinterpret_cast<const uint8_t *>(bm)[r * 64 + lane] : 0u;
            hl[r] = __ballot((hB_[r] >> 31) & 1u);
            lf[r] = __ballot(((lA_[r] & ~spread4(sbits[r])) >> 7) & 1u);
        }

        // one unit of context at each tile end, read only when it matters
        uint64_t carry_in = 0, carry_nx = 0;
        if ((lf[0] & 1ull) && tl - 1 >= lo && !(kSpans && ts.at_tl))
            carry_in = is_high_unit(in[tl - 1]) ? 1ull : 0ull;
        if ((hl[R - 1] >> 63) && th < hi && !(BATCH && ts.next))
            carry_nx = is_low_unit(in[th]) ? 1ull : 0ull;


#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t pm = (hl[r] << 1) | (r == 0 ? carry_in : (hl[r - 1] >> 63));
            const uint64_t nm = (lf[r] >> 1) | ((r == R - 1 ? carry_nx : (lf[r + 1] & 1ull)) << 63);
            const uint32_t hp = (uint32_t)(pm >> lane) & 1u;
            const uint32_t ln = (uint32_t)(nm >> lane) & 1u;
            // Phase 2: mismatches of the row's 8 units
            const uint32_t hA = hA_[r], hB = hB_[r], lA = lA_[r], lB = lB_[r];
            uint32_t badA, badB;
            mismatches(hA, hB, lA, lB, spread4(sbits[r]), spread4(sbits[r] >> 4), hp, ln, badA, badB);
            const bool lane_bad = (badA | badB) != 0u;
            const uint64_t wave_bad = __ballot(lane_bad);
            const int64_t u0 = tl + ((int64_t)r * 64 + lane) * 8;
            const uint64_t bad64 = (uint64_t)badA | ((uint64_t)badB << 32);

            if constexpr (OP == kOpTo) {
                const u32x4 o = wave_bad ? repair(v[r], badA, badB) : v[r];
                if constexpr (SS) {
                    store_shifted<NT>(out, u0, lo, hi, o, prev_lane(o, last, lane), ks, r == 0 && lane == 0,
                                      r == R - 1 && lane == 63);
                    last = lane63(o);
                } else if (interior) {
                    st16<NT>(out + u0, o);
                } else {
                    st_row<NT>(out, tl + (int64_t)r * kRowUnits, lane, lo, hi, o);
                }
            } else if constexpr (OP == kOpToInplace) {
                // Inside the buffer, in the line store mode the eight lanes
                // of a 128-byte line store together when any of them changed,
                // so memory sees whole-line writes rather than partial ones;
                // unchanged lanes write back the values they read, which no
                // other wave writes. In the sector mode (SS) only the lanes
                // that changed store.
                if (interior) {
                    if constexpr (SS) {
                        if (lane_bad)
                            st16<NT>(out + u0, repair(v[r], badA, badB));
                    } else if ((wave_bad >> (lane & ~7)) & 0xFFull) {
                        st16<NT>(out + u0, lane_bad ? repair(v[r], badA, badB) : v[r]);
                    }
                } else if (lane_bad) {
                    st_partial(out, u0, lo, hi, repair(v[r], badA, badB), bad64);
                }
            } else if constexpr (OP == kOpIs) {
                if constexpr (!BATCH) {
                    if (wave_bad) {
                        // Every wave that sees a mismatch clears the result;
                        // the clearing is published with a device-coherent
                        // store (which other waves' polls observe) when it
                        // was found past the wave's first tile, else by one
                        // wave in 256; the rest write through their cache.
                        // Dense errors are found by every wave in its first
                        // tile, at once, and thousands of coherent stores to
                        // one word would queue; but then every wave stops
                        // after that tile anyway. A sparse error is most
                        // likely found past the first tile, and then it is
                        // always published.
                        if (lane == 0 &&
                            __hip_atomic_load(a.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            if (t != tb || (wave & 255) == 0)
                                __hip_atomic_store(a.flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            else
                                __hip_atomic_store(a.flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        return;
                    }
                }
            } else {  // kOpLocate, one buffer
                if (wave_bad) {
                    loc_count += (uint32_t)__popcll(bad64);
                    if (loc_first == ~0ull) {
                        const int fl = __builtin_ctzll(wave_bad);
                        const int j = lane_bad ? (__builtin_ctzll(bad64) >> 3) : 0;
                        const int jf = __shfl(j, fl);
                        loc_first = (uint64_t)(tl + ((int64_t)r * 64 + fl) * 8 + jf - lo);
                    }
                }
            }
        }
    }

    if (OP == kOpLocate && BATCH && !loc_wg) {
        if (loc_k >= 0)
            loc_flush();
    } else if (OP == kOpLocate && BATCH) {
        // The string a wave ends on often spans the whole workgroup (a long
        // string covers thousands of waves): such totals meet in LDS, and
        // the workgroup's last wave adds them with one pair of atomics, not
        // one pair per wave on the same two words (one 2^28-unit string
        // with errors throughout: 241 -> 155 us; the Zipf batch of 4096
        // strings: 498 -> 480 us).
        uint32_t c = loc_count;
#pragma unroll
        for (int sh = 32; sh >= 1; sh >>= 1)
            c += __shfl_xor(c, sh);
        if (lane == 0) {
            if (loc_k >= 0 && c != 0) {
                const unsigned long long kk = (unsigned long long)loc_k;
                const unsigned long long prev = atomicCAS(&s_loc_k, ~0ull, kk);
                if (prev == ~0ull || prev == kk) {
                    atomicAdd(&s_loc_total, (unsigned long long)c);
                    atomicMin(&s_loc_first, (unsigned long long)loc_first);
                } else {
                    atomicAdd(reinterpret_cast<unsigned long long *>(a.count + loc_k), (unsigned long long)c);
                    atomicMin(reinterpret_cast<unsigned long long *>(a.first + loc_k), (unsigned long long)loc_first);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (atomicAdd(&s_loc_done, 1u) == (uint32_t)wg_waves - 1u) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const unsigned long long k = atomicCAS(&s_loc_k, ~0ull, ~0ull);
                const unsigned long long tc = atomicAdd(&s_loc_total, 0ull);
                const unsigned long long tf = atomicMin(&s_loc_first, ~0ull);
                if (k != ~0ull && tc != 0) {
                    atomicAdd(reinterpret_cast<unsigned long long *>(a.count + k), tc);
                    atomicMin(reinterpret_cast<unsigned long long *>(a.first + k), tf);
                }
            }
        }
    }
    if constexpr (kFlatLocate) {
        // wave totals -> workgroup totals in LDS -> one pair of global
        // atomics by the last wave of the workgroup to finish
        uint32_t c = loc_count;
#pragma unroll
        for (int sh = 32; sh >= 1; sh >>= 1)
            c += __shfl_xor(c, sh);
        if (lane == 0) {
            if (c != 0) {
                atomicAdd(&s_loc_count, c);
                atomicMin(&s_loc_first, (unsigned long long)loc_first);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (atomicAdd(&s_loc_done, 1u) == (uint32_t)wg_waves - 1u) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const uint32_t tc = atomicAdd(&s_loc_count, 0u);
                const unsigned long long tf = atomicMin(&s_loc_first, ~0ull);
                if (tc != 0) {
                    atomicAdd(reinterpret_cast<unsigned long long *>(a.count), (unsigned long long)tc);
                    atomicMin(reinterpret_cast<unsigned long long *>(a.first), tf);
                }
            }
        }
    }
}

// isWellFormed of a batch of few, long strings, launched before the main
// pass: one wave per string sets the string's result, to 0 when the string
// has at least kHeadMinUnits units and a mismatch among its first 512 units
// (with the unit after them as context), else to 1 (so no separate clearing
// launch is needed). It lets the main pass skip every tile of a string whose
// first mismatch lies near its start, which that pass cannot learn in time
// on its own: the tiles of one string are all in flight together.
constexpr int64_t kHeadMinUnits = 8192;
__global__ void __launch_bounds__(256) head_check_kernel(const uint16_t *in, const int64_t *off, int64_t nstr,
                                                         int64_t shift, uint8_t *results) {
    const int lane = __lane_id();
    const int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (k >= nstr)
        return;
    const int64_t s0 = off[k] + shift, s1 = off[k + 1] + shift;
    bool clean = true;
    if (s1 - s0 >= kHeadMinUnits) {
        const int64_t hend = s0 + kRowUnits;  // s1 > hend: the head lies inside the string
        const u32x4 v = ld_partial(in, s0 + (int64_t)lane * 8, s0, hend);
        uint32_t hA, hB, lA, lB;
        flags4(high_bytes(v.x, v.y), hA, lA);
        flags4(high_bytes(v.z, v.w), hB, lB);
        const uint64_t hl = __ballot((hB >> 31) & 1u);
        const uint64_t lf = __ballot((lA >> 7) & 1u);
        const uint64_t carry_nx = is_low_unit(in[hend]) ? 1ull : 0ull;  // context only
        const uint32_t hp = (uint32_t)((hl << 1) >> lane) & 1u;           // nothing precedes the string
        const uint32_t ln = (uint32_t)(((lf >> 1) | (carry_nx << 63)) >> lane) & 1u;
        uint32_t badA, badB;
        mismatches(hA, hB, lA, lB, lane == 0 ? 0x80u : 0u, 0u, hp, ln, badA, badB);  // unit s0 starts it
        clean = __ballot((badA | badB) != 0u) == 0ull;
    }
    if (lane == 0)
        results[k] = clean ? 1 : 0;
}

// Separate strings in one launch (the MultiArgs layout): a wave takes a
// contiguous run of the strings' tile numbers and handles each tile as a flat
// call would, with its string's frame; tiles never span two strings.
template <int OP, int R, bool NT>
__global__ void __launch_bounds__(1024) wf_multi_kernel(MultiArgs a) {
    constexpr int64_t T = kRowUnits * R;
    const int lane = __lane_id();
    const int64_t wg_waves = blockDim.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * wg_waves;
    const int64_t wave = (int64_t)blockIdx.x * wg_waves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t per = (a.ntiles + nwaves - 1) / nwaves;
    const int64_t vb = wave * per, ve = min(vb + per, a.ntiles);
    if (vb >= ve)
        return;
    // the string of tile vb: the last one whose first tile is at or before
    // it (of equal tile0, the last is the one that has tiles)
    int i = __popcll(__ballot(lane < a.n && a.s[lane < a.n ? lane : 0].tile0 <= vb)) - 1;
    // check: the result word of string poll_i as read with the previous
    // tile's loads (once it holds the stamp, the string's other tiles are
    // skipped)
    int poll_i = -1;
    uint32_t poll = 0;

    for (int64_t vt = vb; vt < ve; ++vt) {
        while (i + 1 < a.n && a.s[i + 1].tile0 <= vt)
            ++i;
        if constexpr (OP == kOpIs) {
            if (poll_i == i && poll == a.stamp)
                continue;
        }
        const uint16_t *in = a.s[i].in;
        uint16_t *out = a.s[i].out;
        const int64_t lo = a.s[i].lo, hi = a.s[i].hi;
        const int64_t tl = (lo / T + (vt - a.s[i].tile0)) * T, th = tl + T;
        const bool interior = tl >= lo && th <= hi;
        u32x4 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t u0 = tl + ((int64_t)r * 64 + lane) * 8;
            v[r] = interior ? ld16<NT>(in + u0) : ld_row<NT>(in, tl + (int64_t)r * kRowUnits, lane, lo, hi);
        }
        if constexpr (OP == kOpIs) {
            poll = __hip_atomic_load(a.results + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            poll_i = i;
        }
        uint32_t hA_[R], hB_[R], lA_[R], lB_[R];
        uint64_t hl[R], lf[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            flags4(high_bytes(v[r].x, v[r].y), hA_[r], lA_[r]);
            flags4(high_bytes(v[r].z, v[r].w), hB_[r], lB_[r]);
            hl[r] = __ballot((hB_[r] >> 31) & 1u);
            lf[r] = __ballot((lA_[r] >> 7) & 1u);
        }
        uint64_t carry_in = 0, carry_nx = 0;
        if ((lf[0] & 1ull) && tl - 1 >= lo)
            carry_in = is_high_unit(in[tl - 1]) ? 1ull : 0ull;
        if ((hl[R - 1] >> 63) && th < hi)
            carry_nx = is_low_unit(in[th]) ? 1ull : 0ull;
        const bool ss = a.s[i].scalar_store != 0;
        const uint32_t ks = (uint32_t)((reinterpret_cast<uintptr_t>(out) & 15u) >> 1);
        u32x4 last = (u32x4){0u, 0u, 0u, 0u};
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t pm = (hl[r] << 1) | (r == 0 ? carry_in : (hl[r - 1] >> 63));
            const uint64_t nm = (lf[r] >> 1) | ((r == R - 1 ? carry_nx : (lf[r + 1] & 1ull)) << 63);
            uint32_t badA, badB;
            mismatches(hA_[r], hB_[r], lA_[r], lB_[r], 0u, 0u, (uint32_t)(pm >> lane) & 1u,
                       (uint32_t)(nm >> lane) & 1u, badA, badB);
            const uint64_t wave_bad = __ballot((badA | badB) != 0u);
            if constexpr (OP == kOpTo) {
                const int64_t u0 = tl + ((int64_t)r * 64 + lane) * 8;
                const u32x4 o = wave_bad ? repair(v[r], badA, badB) : v[r];
                if (ss) {
                    store_shifted<NT>(out, u0, lo, hi, o, prev_lane(o, last, lane), ks, r == 0 && lane == 0,
                                      r == R - 1 && lane == 63);
                    last = lane63(o);
                } else if (interior) {
                    st16<NT>(out + u0, o);
                } else {
                    st_row<NT>(out, tl + (int64_t)r * kRowUnits, lane, lo, hi, o);
                }
            } else {
                if (wave_bad) {
                    // The stamp is published device-wide by one wave in
                    // sixteen, and only while the string has tiles left for
                    // other waves to skip; the rest store it through their
                    // cache, which the kernel's end writes back. (A coherent
                    // store from every erring tile of a long string queued
                    // on the one word and took the serving loop's check p99
                    // from 63 to 338 us. Waves here often hold one tile, so
                    // the batch check's clean-previous-tile rule would
                    // publish nothing.)
                    if (lane == 0) {
                        if (th < hi && (wave & 15) == 0)
                            __hip_atomic_store(a.results + i, a.stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        else
                            __hip_atomic_store(a.results + i, a.stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    poll = a.stamp;
                    break;
                }
            }
        }
    }
}

// Plain copy with the same tiling: the bandwidth ceiling for the repair.
template <int R, bool NT>
__global__ void __launch_bounds__(1024) copy_kernel(const uint16_t *in, uint16_t *out, int64_t lo, int64_t hi) {
    constexpr int64_t T = kRowUnits * R;
    const int lane = __lane_id();
    const int64_t wg_waves = blockDim.x >> 6;
    const int64_t nwaves = (int64_t)gridDim.x * wg_waves;
    const int64_t wave = (int64_t)blockIdx.x * wg_waves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (hi <= lo)
        return;
    const int64_t t0 = lo / T, t1 = (hi + T - 1) / T;
    const int64_t per = (t1 - t0 + nwaves - 1) / nwaves;
    const int64_t tb = t0 + wave * per;
    const int64_t te = min(tb + per, t1);
    for (int64_t t = tb; t < te; ++t) {
        const int64_t tl = t * T;
        const bool interior = tl >= lo && tl + T <= hi;
        u32x4 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t u0 = tl + ((int64_t)r * 64 + lane) * 8;
            v[r] = interior ? ld16<NT>(in + u0) : ld_row<NT>(in, tl + (int64_t)r * kRowUnits, lane, lo, hi);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t u0 = tl + ((int64_t)r * 64 + lane) * 8;
            if (interior)
                st16<NT>(out + u0, v[r]);
            else
                st_row<NT>(out, tl + (int64_t)r * kRowUnits, lane, lo, hi, v[r]);
        }
    }
}

// Fills up to two byte ranges (blockIdx.y picks one) with a repeating
// 16-byte pattern: byte a of memory gets byte (a mod 16) of the pattern. A
// range that starts on an element boundary of an element size dividing 16
// thus holds the element value repeated. The 16-byte-aligned body is written
// with vector stores, the unaligned head and tail byte by byte.
struct FillRange {
    uint8_t *p;
    int64_t nbytes;
    u32x4 pat;
};
__device__ __forceinline__ uint8_t pattern_byte(u32x4 pat, uint32_t k) {
    const uint32_t d = k < 4 ? pat.x : k < 8 ? pat.y : k < 12 ? pat.z : pat.w;
    return (uint8_t)(d >> (8 * (k & 3)));
}
__global__ void __launch_bounds__(256) fill_kernel(FillRange r0, FillRange r1) {
    const FillRange &r = blockIdx.y == 0 ? r0 : r1;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(r.p);
    const int64_t head = min(r.nbytes, (int64_t)((16u - (a0 & 15u)) & 15u));
    const int64_t nv = (r.nbytes - head) >> 4;
    const int64_t tail = head + nv * 16;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    u32x4 *q = reinterpret_cast<u32x4 *>(r.p + head);
    for (int64_t i = gid; i < nv; i += stride)
        q[i] = r.pat;
    if (gid < head)
        r.p[gid] = pattern_byte(r.pat, (uint32_t)((a0 + gid) & 15u));
    if (gid < r.nbytes - tail)
        r.p[tail + gid] = pattern_byte(r.pat, (uint32_t)((a0 + tail + gid) & 15u));
}

__global__ void validate_kernel(const int64_t *off, int64_t nstr, int64_t buf_units, int32_t *bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nstr; i += stride) {
        const int64_t o = off[i];
        bool ok = o >= 0 && o <= buf_units;
        if (i < nstr)
            ok = ok && off[i + 1] >= o;
        if (!ok)
            *bad = 1;
    }
}

__device__ void copy_chunk(const CopyChunk &c);

// Copies each chunk (one workgroup per chunk) with 16-byte stores: after a
// head that aligns the destination, each 16-byte destination vector is built
// from the two aligned 16-byte source vectors it straddles (when source and
// destination alignments differ) or copied straight (when they agree). Only
// the last vector and the tail go unit by unit, so no source byte past the
// chunk is ever read.
__global__ void __launch_bounds__(256) chunk_copy_kernel(const CopyChunk *chunks) {
    copy_chunk(chunks[blockIdx.x]);
}

__device__ void copy_chunk(const CopyChunk &c) {
    const int64_t n = c.n;
    const uintptr_t sa = reinterpret_cast<uintptr_t>(c.src), da = reinterpret_cast<uintptr_t>(c.dst);
    const int64_t head = min(n, (int64_t)(((16u - (da & 15u)) & 15u) >> 1));
    if (threadIdx.x < head)
        c.dst[threadIdx.x] = c.src[threadIdx.x];
    const int64_t nv = (n - head) >> 3;  // whole destination vectors
    u32x4 *d4 = reinterpret_cast<u32x4 *>(c.dst + head);
    int64_t done = head;                 // units [0, done) handled by the vector loops
    if (((sa ^ da) & 15u) == 0) {
        const u32x4 *s4 = reinterpret_cast<const u32x4 *>(c.src + head);
        for (int64_t i = threadIdx.x; i < nv; i += blockDim.x)
            d4[i] = s4[i];
        done = head + nv * 8;
    } else if (nv >= 2) {
        const uintptr_t s0 = sa + 2 * (uintptr_t)head;
        const u32x4 *sv = reinterpret_cast<const u32x4 *>(s0 & ~(uintptr_t)15);
        const uint32_t sh = (uint32_t)(s0 & 15u);
        // vector i reads source vectors i and i+1; for i <= nv - 2 both end
        // at or before the source byte of unit head + 8 * nv <= n
        for (int64_t i = threadIdx.x; i < nv - 1; i += blockDim.x)
            d4[i] = realign(sv[i], sv[i + 1], sh);
        done = head + (nv - 1) * 8;
    }
    for (int64_t i = done + threadIdx.x; i < n; i += blockDim.x)
        c.dst[i] = c.src[i];
}

// The 16-byte pattern of element value v (size 1, 4 or 8 bytes).
template <typename T>
FillRange fill_range(T *p, T v, int64_t n) {
    static_assert(16 % sizeof(T) == 0, "element size must divide 16");
    FillRange r;
    r.p = reinterpret_cast<uint8_t *>(p);
    r.nbytes = n > 0 ? n * (int64_t)sizeof(T) : 0;
    uint32_t w[4];
    uint8_t *b = reinterpret_cast<uint8_t *>(w);
    for (int i = 0; i < 16; ++i)
        b[i] = reinterpret_cast<const uint8_t *>(&v)[i % sizeof(T)];
    r.pat = (u32x4){w[0], w[1], w[2], w[3]};
    return r;
}

hipError_t fill2(const FillRange &r0, const FillRange &r1, hipStream_t s) {
    const int64_t nb = max(r0.nbytes, r1.nbytes);
    if (nb <= 0)
        return hipSuccess;
    // one 16-byte store per thread, at most 2048 workgroups per range
    const int64_t blocks = max((int64_t)1, min((nb / 16 + 255) / 256, (int64_t)2048));
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks, r1.nbytes > 0 ? 2u : 1u), dim3(256), 0, s, r0, r1);
    return hipGetLastError();
}

template <typename T>
hipError_t fill(T *p, T v, int64_t n, hipStream_t s) {
    return fill2(fill_range(p, v, n), FillRange{nullptr, 0, (u32x4){0, 0, 0, 0}}, s);
}

template <int OP, bool BATCH, int R, bool NT>
hipError_t launch_r(const LaunchShape &sh, const KernelArgs &a, hipStream_t s) {
    const dim3 grid((unsigned)sh.grid), block((unsigned)(64 * sh.wg_waves));
    bool alt = false;  // the SS variant: realigned stores, or sector stores in place
    if constexpr (OP == kOpTo)
        alt = a.scalar_store != 0;
    else if constexpr (OP == kOpToInplace)
        alt = sh.store_lines == 0;
    if constexpr (OP == kOpTo || OP == kOpToInplace) {
        if (alt) {
            hipLaunchKernelGGL((wf_kernel<OP, BATCH, R, NT, true>), grid, block, 0, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((wf_kernel<OP, BATCH, R, NT, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int OP, bool BATCH>
hipError_t launch_ob(const LaunchShape &sh, const KernelArgs &a, hipStream_t s) {
    const bool nt = sh.nontemporal != 0;
    switch (sh.rows) {
    case 1: return nt ? launch_r<OP, BATCH, 1, true>(sh, a, s) : launch_r<OP, BATCH, 1, false>(sh, a, s);
    case 2: return nt ? launch_r<OP, BATCH, 2, true>(sh, a, s) : launch_r<OP, BATCH, 2, false>(sh, a, s);
    case 4: return nt ? launch_r<OP, BATCH, 4, true>(sh, a, s) : launch_r<OP, BATCH, 4, false>(sh, a, s);
    case 8: return nt ? launch_r<OP, BATCH, 8, true>(sh, a, s) : launch_r<OP, BATCH, 8, false>(sh, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool BATCH>
hipError_t launch_b(int op, const LaunchShape &sh, const KernelArgs &a, hipStream_t s) {
    switch (op) {
    case kOpIs: return launch_ob<kOpIs, BATCH>(sh, a, s);
    case kOpTo: return launch_ob<kOpTo, BATCH>(sh, a, s);
    case kOpToInplace: return launch_ob<kOpToInplace, BATCH>(sh, a, s);
    case kOpLocate: return launch_ob<kOpLocate, BATCH>(sh, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int R>
hipError_t launch_copy_r(const uint16_t *in, uint16_t *out, int64_t lo, int64_t hi, const LaunchShape &sh,
                         hipStream_t s) {
    const dim3 grid((unsigned)sh.grid), block((unsigned)(64 * sh.wg_waves));
    if (sh.nontemporal)
        hipLaunchKernelGGL((copy_kernel<R, true>), grid, block, 0, s, in, out, lo, hi);
    else
        hipLaunchKernelGGL((copy_kernel<R, false>), grid, block, 0, s, in, out, lo, hi);
    return hipGetLastError();
}

template <int OP, int R>
hipError_t launch_multi_r(const LaunchShape &sh, const MultiArgs &a, hipStream_t s) {
    const dim3 grid((unsigned)sh.grid), block((unsigned)(64 * sh.wg_waves));
    if (sh.nontemporal)
        hipLaunchKernelGGL((wf_multi_kernel<OP, R, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((wf_multi_kernel<OP, R, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <int OP>
hipError_t launch_multi_op(const LaunchShape &sh, const MultiArgs &a, hipStream_t s) {
    switch (sh.rows) {
    case 1: return launch_multi_r<OP, 1>(sh, a, s);
    case 2: return launch_multi_r<OP, 2>(sh, a, s);
    case 4: return launch_multi_r<OP, 4>(sh, a, s);
    case 8: return launch_multi_r<OP, 8>(sh, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_main(int op, bool batch, const LaunchShape &shape, const KernelArgs &a, hipStream_t stream) {
    return batch ? launch_b<true>(op, shape, a, stream) : launch_b<false>(op, shape, a, stream);
}

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s) { return fill<uint8_t>(p, v, n, s); }
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) { return fill<int32_t>(p, v, n, s); }
hipError_t launch_fill_locate(int64_t *first, int64_t *count, int64_t n, hipStream_t s) {
    return fill2(fill_range(first, (int64_t)-1, n), fill_range(count, (int64_t)0, n), s);
}

hipError_t launch_copy(const uint16_t *in, uint16_t *out, int64_t lo, int64_t hi, const LaunchShape &shape,
                       hipStream_t s) {
    switch (shape.rows) {
    case 1: return launch_copy_r<1>(in, out, lo, hi, shape, s);
    case 2: return launch_copy_r<2>(in, out, lo, hi, shape, s);
    case 4: return launch_copy_r<4>(in, out, lo, hi, shape, s);
    case 8: return launch_copy_r<8>(in, out, lo, hi, shape, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_chunk_copy(const CopyChunk *chunks, int64_t nchunks, hipStream_t s) {
    if (nchunks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(chunk_copy_kernel, dim3((unsigned)nchunks), dim3(256), 0, s, chunks);
    return hipGetLastError();
}

hipError_t launch_multi(int op, const LaunchShape &shape, const MultiArgs &a, hipStream_t s) {
    if (a.ntiles <= 0 || a.n <= 0)
        return hipSuccess;
    if (a.n > kMultiMax)
        return hipErrorInvalidValue;
    switch (op) {
    case kOpTo: return launch_multi_op<kOpTo>(shape, a, s);
    case kOpIs: return launch_multi_op<kOpIs>(shape, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_head_check(const uint16_t *in_frame, const int64_t *offsets, int64_t nstr, int64_t shift,
                             uint8_t *results, hipStream_t s) {
    if (nstr <= 0)
        return hipSuccess;
    const int64_t blocks = (nstr + 3) / 4;
    hipLaunchKernelGGL(head_check_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in_frame, offsets, nstr, shift,
                       results);
    return hipGetLastError();
}

hipError_t launch_validate(const int64_t *offsets, int64_t nstr, int64_t buf_units, int32_t *bad, hipStream_t s) {
    const int64_t blocks = min((nstr + 1 + 255) / 256, (int64_t)4096);
    hipLaunchKernelGGL(validate_kernel, dim3((unsigned)blocks), dim3(256), 0, s, offsets, nstr, buf_units, bad);
    return hipGetLastError();
}

}  // namespace utf16wf
