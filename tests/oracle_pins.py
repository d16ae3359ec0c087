"""Checks that pin the CPU oracle to facts fixed outside the oracle itself.

Each pin takes an ``impl`` (an ``OracleLib`` around a compiled oracle) so the
mutation test can run the same pins against deliberately broken builds of the
oracle source and show that every planted mistake is caught.

What pins the oracle:
  * the worked example printed in the paper (Sec. 3.1, Fig. 3);
  * Python's own UTF-16 codec with ``errors='replace'`` (a library routine
    that replaces each unpaired surrogate unit with U+FFFD);
  * the paper's block formulation (Sec. 3.1): a unit is mismatched when it is
    a high surrogate whose successor is not a low one, or a low surrogate
    whose predecessor is not a high one, with out-of-range neighbours counting
    as non-surrogates. Equality with the sequential walk is a theorem
    (locality), checked exhaustively on short strings and on every window of
    top-6-bit classes;
  * the code-point formula of Sec. 1, used to decode and re-encode;
  * invariants: well-formed output, same length, only surrogates change and
    they become U+FFFD, idempotence, fixed points, slicing, in-place = copy.
"""
from __future__ import annotations

import ctypes
import itertools
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
REPL = 0xFFFD


# ------------------------------------------------------------------ helpers

def load_fig3():
    path = os.path.join(HERE, "golden", "fig3_example.txt")
    rows = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows[key] = np.array([int(v, 16) for v in vals], dtype=np.uint16)
    return rows["input"], rows["output"]


def codec_repair(s) -> np.ndarray:
    """CPython's UTF-16 decoder with replacement, re-encoded."""
    b = np.ascontiguousarray(s, dtype=np.uint16).tobytes()
    return np.frombuffer(b.decode("utf-16-le", "replace").encode("utf-16-le"), dtype=np.uint16)


def codec_strict_ok(s) -> bool:
    try:
        np.ascontiguousarray(s, dtype=np.uint16).tobytes().decode("utf-16-le", "strict")
        return True
    except UnicodeDecodeError:
        return False


def block_rule(s, starts=None) -> np.ndarray:
    """Paper's block formulation (Sec. 3.1), vectorised over a whole array:
    mismatched = (high & next not low) | (low & previous not high). ``starts``
    (bool per unit) marks string starts in a packed batch: no pairing across
    them."""
    s = np.asarray(s, dtype=np.uint16)
    top = s & 0xFC00
    hi = top == 0xD800
    lo = top == 0xDC00
    prev_hi = np.zeros_like(hi)
    prev_hi[1:] = hi[:-1]
    next_lo = np.zeros_like(lo)
    next_lo[:-1] = lo[1:]
    if starts is not None:
        prev_hi &= ~starts
        cut_next = np.zeros_like(lo)
        cut_next[:-1] = starts[1:]
        next_lo &= ~cut_next
    bad = (hi & ~next_lo) | (lo & ~prev_hi)
    out = s.copy()
    out[bad] = REPL
    return out


def decode_codepoints(s):
    """Code points of a well-formed UTF-16 array via the Sec. 1 formula."""
    s = [int(x) for x in s]
    cps, i = [], 0
    while i < len(s):
        u = s[i]
        if 0xD800 <= u <= 0xDBFF:
            lo = s[i + 1]
            assert 0xDC00 <= lo <= 0xDFFF, "not well-formed"
            cps.append(((u - 0xD800) << 10) + (lo - 0xDC00) + 0x10000)
            i += 2
        else:
            assert not (0xDC00 <= u <= 0xDFFF), "not well-formed"
            cps.append(u)
            i += 1
    return cps


def encode_codepoints(cps):
    out = []
    for c in cps:
        if c >= 0x10000:
            v = c - 0x10000
            out += [0xD800 + (v >> 10), 0xDC00 + (v & 0x3FF)]
        else:
            out.append(c)
    return np.array(out, dtype=np.uint16)


class OracleLib:
    """Thin wrapper over a compiled oracle (real or mutant)."""

    def __init__(self, path):
        lib = ctypes.CDLL(path)
        p, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.wf_to_seq.argtypes = [p, p, i64]
        lib.wf_to_seq.restype = i64
        lib.wf_is_seq.argtypes = [p, i64]
        lib.wf_is_seq.restype = ctypes.c_int
        lib.wf_first_bad_seq.argtypes = [p, i64]
        lib.wf_first_bad_seq.restype = i64
        lib.wf_to_batch.argtypes = [p, p, p, i64]
        lib.wf_to_batch.restype = i64
        lib.wf_is_batch.argtypes = [p, p, i64, p]
        lib.wf_is_batch.restype = None
        lib.wf_locate_batch.argtypes = [p, p, i64, p, p]
        lib.wf_locate_batch.restype = None
        lib.wf_to_chunked_mt.argtypes = [p, p, i64, ctypes.c_int]
        lib.wf_to_chunked_mt.restype = i64
        self.lib = lib

    @staticmethod
    def _a(s):
        return np.ascontiguousarray(s, dtype=np.uint16)

    def to(self, s):
        s = self._a(s)
        t = np.empty_like(s)
        self.lib.wf_to_seq(s.ctypes.data, t.ctypes.data, s.size)
        return t

    def to_count(self, s):
        s = self._a(s)
        t = np.empty_like(s)
        c = self.lib.wf_to_seq(s.ctypes.data, t.ctypes.data, s.size)
        return t, int(c)

    def to_inplace(self, s):
        t = self._a(s).copy()
        self.lib.wf_to_seq(t.ctypes.data, t.ctypes.data, t.size)
        return t

    def is_(self, s):
        s = self._a(s)
        return bool(self.lib.wf_is_seq(s.ctypes.data, s.size))

    def first_bad(self, s):
        s = self._a(s)
        return int(self.lib.wf_first_bad_seq(s.ctypes.data, s.size))

    def to_batch(self, buf, off, fill=None):
        buf = self._a(buf)
        off = np.ascontiguousarray(off, dtype=np.int64)
        t = buf.copy() if fill is None else self._a(fill).copy()
        self.lib.wf_to_batch(buf.ctypes.data, t.ctypes.data, off.ctypes.data, off.size - 1)
        return t

    def is_batch(self, buf, off):
        buf = self._a(buf)
        off = np.ascontiguousarray(off, dtype=np.int64)
        r = np.empty(off.size - 1, dtype=np.uint8)
        self.lib.wf_is_batch(buf.ctypes.data, off.ctypes.data, off.size - 1, r.ctypes.data)
        return r

    def locate_batch(self, buf, off):
        buf = self._a(buf)
        off = np.ascontiguousarray(off, dtype=np.int64)
        b = off.size - 1
        first = np.empty(b, dtype=np.int64)
        cnt = np.empty(b, dtype=np.int64)
        self.lib.wf_locate_batch(buf.ctypes.data, off.ctypes.data, b, first.ctypes.data, cnt.ctypes.data)
        return first, cnt

    def to_mt(self, s, threads):
        s = self._a(s)
        t = np.empty_like(s)
        r = self.lib.wf_to_chunked_mt(s.ctypes.data, t.ctypes.data, s.size, int(threads))
        assert r >= 0
        return t


# ------------------------------------------------------------- the pins

CLASS_REPS = (0x0041, 0x4E2D, 0xD83D, 0xDE0A)  # ASCII, BMP, high, low
EDGE_ALPHABET = (0x0000, 0x007F, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xE000, 0xFFFD, 0xFFFF)


def pin_fig3(impl):
    inp, out = load_fig3()
    assert inp.size == 31
    assert np.array_equal(impl.to(inp), out)
    assert not impl.is_(inp)
    assert impl.first_bad(inp) == 10
    # Fig. 3 pads the string with U+0000 on both sides; padding changes nothing.
    padded = np.concatenate([[0], inp, [0]]).astype(np.uint16)
    assert np.array_equal(impl.to(padded)[1:-1], out)


def _all_sequences(alphabet, max_len):
    for n in range(0, max_len + 1):
        for seq in itertools.product(alphabet, repeat=n):
            yield np.array(seq, dtype=np.uint16)


def pin_codec_bruteforce(impl, max_len=4):
    """Every sequence of length 0..4 over the class representatives and over
    the edge alphabet equals the codec's repair; ``is`` agrees with strict
    decoding; the count of replaced units matches."""
    for alphabet in (CLASS_REPS, EDGE_ALPHABET):
        for s in _all_sequences(alphabet, max_len):
            want = codec_repair(s)
            got, cnt = impl.to_count(s)
            assert np.array_equal(got, want), (s, got, want)
            assert impl.is_(s) == codec_strict_ok(s), s
            assert cnt == int(np.count_nonzero(want != s)), s


def pin_block_rule_short(impl, max_len=8):
    """Sequential walk == block formulation for all 4-class strings up to 8."""
    rng = np.random.default_rng(7)
    for s in _all_sequences(CLASS_REPS, max_len):
        # vary the low bits so the classes are not a single value each
        s = s ^ (rng.integers(0, 1024, size=s.size) & 0x3FF).astype(np.uint16) * (s >= 0xD800)
        assert np.array_equal(impl.to(s), block_rule(s)), s


def pin_windows_exhaustive(impl, seed=11):
    """All 64^3 windows of top-6-bit classes (random low 10 bits), each window
    isolated by ASCII on both sides, in one long string: the middle unit of
    every window must follow the block formulation, so the unit's output
    depends on its two neighbours only."""
    rng = np.random.default_rng(seed)
    cls = np.arange(64, dtype=np.uint32)
    a, b, c = np.meshgrid(cls, cls, cls, indexing="ij")
    win = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)
    units = (win << 10) | rng.integers(0, 1024, size=win.shape).astype(np.uint32)
    s = np.full((win.shape[0], 4), 0x0041, dtype=np.uint32)
    s[:, :3] = units
    s = s.ravel().astype(np.uint16)
    assert np.array_equal(impl.to(s), block_rule(s))
    assert np.array_equal(impl.to(s), codec_repair(s))


def pin_random_vs_codec(impl, seed=3, cases=3000):
    rng = np.random.default_rng(seed)
    alphabet = np.array(EDGE_ALPHABET + CLASS_REPS, dtype=np.uint16)
    for _ in range(cases):
        n = int(rng.integers(0, 40))
        s = alphabet[rng.integers(0, alphabet.size, size=n)]
        s = s ^ ((s >= 0xD800) & (s <= 0xDFFF)) * rng.integers(0, 1024, size=n).astype(np.uint16)
        want = codec_repair(s)
        assert np.array_equal(impl.to(s), want), s
        assert np.array_equal(impl.to_inplace(s), want), s
        fb = impl.first_bad(s)
        diff = np.nonzero(want != s)[0]
        assert fb == (int(diff[0]) if diff.size else -1), s


def pin_batch(impl, seed=5, cases=400):
    """Per-string repair of a packed batch == the codec on every string alone,
    including empty strings and pairs split by a string boundary; units
    outside [off[0], off[B]) are left alone."""
    rng = np.random.default_rng(seed)
    alphabet = np.array([0x41, 0x4E2D, 0xD800, 0xDBFF, 0xDC00, 0xDFFF], dtype=np.uint16)
    for _ in range(cases):
        b = int(rng.integers(0, 12))
        lens = rng.integers(0, 6, size=b)
        pre, post = int(rng.integers(0, 3)), int(rng.integers(0, 3))
        total = int(lens.sum()) + pre + post
        buf = alphabet[rng.integers(0, alphabet.size, size=total)]
        off = np.concatenate([[pre], pre + np.cumsum(lens)]).astype(np.int64)
        fill = np.full(total, 0x1234, dtype=np.uint16)
        got = impl.to_batch(buf, off, fill=fill)
        assert np.all(got[:pre] == 0x1234) and np.all(got[off[-1]:] == 0x1234)
        res = impl.is_batch(buf, off)
        first, cnt = impl.locate_batch(buf, off)
        for k in range(b):
            piece = buf[off[k]:off[k + 1]]
            want = codec_repair(piece)
            assert np.array_equal(got[off[k]:off[k + 1]], want)
            assert res[k] == int(codec_strict_ok(piece))
            diff = np.nonzero(want != piece)[0]
            assert first[k] == (int(diff[0]) if diff.size else -1)
            assert cnt[k] == diff.size
    # a pair cut by a boundary is two lone surrogates
    buf = np.array([0xD800, 0xDC00], dtype=np.uint16)
    assert np.array_equal(impl.to_batch(buf, [0, 1, 2]), [REPL, REPL])
    assert np.array_equal(impl.to_batch(buf, [0, 2]), buf)


def pin_chunked(impl, seed=9):
    """Chunked multi-threaded walk == codec, with chunk edges that split pairs."""
    rng = np.random.default_rng(seed)
    for n in (1, 2, 3, 7, 16, 33, 1000):
        for _ in range(20):
            s = rng.choice(np.array([0x41, 0xD800, 0xDC00, 0xDBFF, 0xDFFF], dtype=np.uint16), size=n)
            want = codec_repair(s)
            for th in (1, 2, 3, 5, 8, 17):
                assert np.array_equal(impl.to_mt(s, th), want), (n, th)


ALL_PINS = (pin_fig3, pin_codec_bruteforce, pin_block_rule_short, pin_windows_exhaustive,
            pin_random_vs_codec, pin_batch, pin_chunked)
