"""Seeded synthetic UTF-16 inputs shared by the tests, the benchmark and the oracle.

This module only draws code units; it holds none of the repair method's
arithmetic (no classification of units, no pairing, no replacement). Every
array is host ``numpy.uint16`` (little-endian code units) and every size or
offsets array is ``numpy.int64``. The same (function, arguments, seed) always
gives the same bytes.

Character mix (``mix``): each *character slot* is, independently,
  - a lone surrogate with probability ``r`` (high or low with equal odds,
    value uniform over 0xD800..0xDBFF or 0xDC00..0xDFFF);
  - otherwise ASCII 0x20..0x7E, a BMP non-surrogate unit (uniform over
    0x0080..0xD7FF and 0xE000..0xFFFF), or a valid pair (high 0xD800..0xDBFF
    then low 0xDC00..0xDFFF) with weights 90 : 7.9 : 2.
At r = 1e-3 this is 90 / 7.9 / 2 / 0.1 percent of slots. A pair that would not
fit in the last unit becomes ASCII. Lone surrogates that happen to land next to
each other may form a valid pair; the repair, not the generator, decides what
is well-formed. The paper's generator works the same way (Sec. 4: a share of
characters are pairs, a share of the other units are lone surrogates, chosen
high or low with equal odds, and accidental pairs are tolerated).
"""
from __future__ import annotations

import math

import numpy as np

ASCII = 0
BMP = 1
PAIR = 2
LONE = 3

_U32 = float(1 << 32)

# Fixed seeds per workload and variant.
SEEDS = {
    "small": 1001,
    "single_ascii": 1101,
    "single_mix0": 1102,
    "single_mix1e-6": 1103,
    "single_mix1e-2": 1104,
    "single_allsur": 1105,
    "ragged_1m": 1201,
    "small_batch": 1204,
    "zipf_4096": 1301,
    "serve": 1401,
    "paper_1m": 1501,
    "paper_sweep": 1502,
    "js_1024": 1503,
}


def _rng(seed) -> np.random.Generator:
    return seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)


def _bmp_values(rng, k):
    """k values uniform over the 63,360 BMP non-surrogate units >= 0x80."""
    v = rng.integers(0, 63360, size=k, dtype=np.int32) + 0x80
    v = v + (v >= 0xD800) * 0x800  # skip the 2048 surrogate values
    return v.astype(np.uint16)


def _fill_slots(n, cats, rng):
    """Write units for slot categories ``cats`` into a fresh array of n units."""
    widths = np.where(cats == PAIR, 2, 1).astype(np.int64)
    starts = np.cumsum(widths) - widths
    keep = starts < n
    cats = cats[keep]
    starts = starts[keep]
    if cats.size and cats[-1] == PAIR and starts[-1] == n - 1:
        cats = cats.copy()
        cats[-1] = ASCII
    out = np.empty(n, dtype=np.uint16)
    pos = starts[cats == ASCII]
    out[pos] = rng.integers(0x20, 0x7F, size=pos.size, dtype=np.int32).astype(np.uint16)
    pos = starts[cats == BMP]
    out[pos] = _bmp_values(rng, pos.size)
    pos = starts[cats == PAIR]
    out[pos] = (0xD800 + rng.integers(0, 1024, size=pos.size, dtype=np.int32)).astype(np.uint16)
    out[pos + 1] = (0xDC00 + rng.integers(0, 1024, size=pos.size, dtype=np.int32)).astype(np.uint16)
    pos = starts[cats == LONE]
    hi = rng.integers(0, 2, size=pos.size, dtype=np.int32)
    out[pos] = (np.where(hi == 1, 0xD800, 0xDC00)
                + rng.integers(0, 1024, size=pos.size, dtype=np.int32)).astype(np.uint16)
    return out


def mix(n: int, r: float, seed) -> np.ndarray:
    """n code units of the character mix above with lone-surrogate rate r."""
    n = int(n)
    if n <= 0:
        return np.empty(0, dtype=np.uint16)
    rng = _rng(seed)
    w = (1.0 - r) / 0.999
    p_lone, p_pair, p_bmp = r, 0.02 * w, 0.079 * w
    t_lone = np.uint32(min(p_lone * _U32, _U32 - 1))
    t_pair = np.uint32(min((p_lone + p_pair) * _U32, _U32 - 1))
    t_bmp = np.uint32(min((p_lone + p_pair + p_bmp) * _U32, _U32 - 1))
    u = rng.integers(0, 1 << 32, size=n, dtype=np.uint32)
    cats = np.full(n, ASCII, dtype=np.uint8)
    cats[u < t_bmp] = BMP
    cats[u < t_pair] = PAIR
    cats[u < t_lone] = LONE
    del u
    return _fill_slots(n, cats, rng)


def ascii_units(n: int, seed) -> np.ndarray:
    return _rng(seed).integers(0x20, 0x7F, size=int(n), dtype=np.int32).astype(np.uint16)


def all_surrogates(n: int, seed) -> np.ndarray:
    """Every unit uniform over 0xD800..0xDFFF (the worst case)."""
    return _rng(seed).integers(0xD800, 0xE000, size=int(n), dtype=np.int32).astype(np.uint16)


# ---------------------------------------------------------------- workloads

SMALL_N = 1 << 20
SINGLE_N = 1 << 28
SINGLE_VARIANTS = ("ascii", "mix0", "mix1e-6", "mix1e-2", "allsur")


def small_string(seed=SEEDS["small"], n=SMALL_N) -> np.ndarray:
    """1,048,576 units of mix(r=1e-3) with a lone low forced at index 0 and a
    lone high forced at the last index."""
    rng = _rng(seed)
    s = mix(n, 1e-3, rng)
    s[0] = 0xDC00 + int(rng.integers(0, 1024))
    s[-1] = 0xD800 + int(rng.integers(0, 1024))
    return s


def single_buffer(variant: str, n=SINGLE_N, seed=None) -> np.ndarray:
    """One of the five 512 MiB single-buffer variants (n units)."""
    if seed is None:
        seed = SEEDS["single_" + variant]
    if variant == "ascii":
        return ascii_units(n, seed)
    if variant == "mix0":
        return mix(n, 0.0, seed)
    if variant == "mix1e-6":
        return mix(n, 1e-6, seed)
    if variant == "mix1e-2":
        return mix(n, 1e-2, seed)
    if variant == "allsur":
        return all_surrogates(n, seed)
    raise ValueError(f"unknown single-buffer variant {variant!r}")


def lognormal_lengths(b: int, rng, median=32.0, sigma=1.5, lo=1, hi=65536) -> np.ndarray:
    z = rng.standard_normal(b)
    return np.clip(np.rint(np.exp(math.log(median) + sigma * z)), lo, hi).astype(np.int64)


def offsets_from_lengths(lengths, base: int = 0) -> np.ndarray:
    off = np.empty(len(lengths) + 1, dtype=np.int64)
    off[0] = base
    np.cumsum(lengths, out=off[1:])
    off[1:] += base
    return off


def ragged_batch(b=1_000_000, seed=SEEDS["ragged_1m"], edge_p=0.05, r=1e-3, median=32.0):
    """(buf, offsets): b strings with log-normal lengths (median ``median``,
    sigma 1.5, clamped to 1..65,536) cut from one mix(r) stream; each string's
    last unit is forced to a lone high and its first unit to a lone low,
    independently with probability ``edge_p`` each."""
    rng = _rng(seed)
    lens = lognormal_lengths(b, rng, median=median)
    off = offsets_from_lengths(lens)
    buf = mix(int(off[-1]), r, rng)
    ends = off[1:][rng.random(b) < edge_p] - 1
    buf[ends] = (0xD800 + rng.integers(0, 1024, size=ends.size)).astype(np.uint16)
    starts = off[:-1][rng.random(b) < edge_p]
    buf[starts] = (0xDC00 + rng.integers(0, 1024, size=starts.size)).astype(np.uint16)
    return buf, off


def small_batch():
    """A serving-size batch: 32 strings of the log-normal batch's shape at
    median 1024 units (about 10^5 units in all)."""
    return ragged_batch(b=32, seed=SEEDS["small_batch"], median=1024.0)


def zipf_lengths(b: int, rng, s=1.1, max_len=1 << 24) -> np.ndarray:
    """i.i.d. lengths from the Zipf(s) law truncated to 1..max_len, by exact
    inverse CDF over the full table."""
    k = np.arange(1, max_len + 1, dtype=np.float64)
    cdf = np.cumsum(k ** (-s))
    cdf /= cdf[-1]
    u = rng.random(b)
    return (np.searchsorted(cdf, u, side="left") + 1).astype(np.int64)


def zipf_batch(b=4096, seed=SEEDS["zipf_4096"], max_len=1 << 24, r=1e-2):
    """(buf, offsets, is_error_string): b strings with Zipf(1.1) lengths over
    1..max_len; each string is, by a seeded coin, pure ASCII or mix(r). String
    contents are slices at seeded offsets of one ASCII pool and one mix(r)
    pool of max_len units each."""
    rng = _rng(seed)
    lens = zipf_lengths(b, rng, max_len=max_len)
    kind = rng.integers(0, 2, size=b).astype(bool)
    pool_len = int(max_len)
    pool_a = ascii_units(pool_len, rng)
    pool_m = mix(pool_len, r, rng)
    off = offsets_from_lengths(lens)
    buf = np.empty(int(off[-1]), dtype=np.uint16)
    starts = rng.integers(0, pool_len - lens + 1)
    for k in range(b):
        src = pool_m if kind[k] else pool_a
        buf[off[k]:off[k + 1]] = src[starts[k]:starts[k] + lens[k]]
    return buf, off, kind


def paper_mix(n: int, pair_pct: float, mis_pct: float, seed) -> np.ndarray:
    """The paper's generator shape (Sec. 4): ``pair_pct`` percent of characters
    are valid pairs; ``mis_pct`` percent of the other units are lone
    surrogates (high or low with equal odds); the remaining units follow the
    ASCII : BMP weights of ``mix`` (90 : 7.9)."""
    n = int(n)
    rng = _rng(seed)
    p_pair = pair_pct / 100.0
    p_lone = (1.0 - p_pair) * mis_pct / 100.0
    rest = 1.0 - p_pair - p_lone
    p_bmp = rest * 0.079 / 0.979
    u = rng.integers(0, 1 << 32, size=max(n, 0), dtype=np.uint32)
    cats = np.full(u.size, ASCII, dtype=np.uint8)
    cats[u < np.uint32(min((p_lone + p_pair + p_bmp) * _U32, _U32 - 1))] = BMP
    cats[u < np.uint32(min((p_lone + p_pair) * _U32, _U32 - 1))] = PAIR
    cats[u < np.uint32(min(p_lone * _U32, _U32 - 1))] = LONE
    if n <= 0:
        return np.empty(0, dtype=np.uint16)
    return _fill_slots(n, cats, rng)


def js_string(n=1024, seed=SEEDS["js_1024"], low_pct=5.0, high_pct=5.0) -> np.ndarray:
    """The JavaScript benchmark shape (Sec. 4.1, Fig. 1): each unit is a low
    surrogate with 5 %, a high surrogate with 5 %, otherwise ASCII."""
    rng = _rng(seed)
    u = rng.random(n)
    s = rng.integers(0x20, 0x7F, size=n, dtype=np.int32)
    lo = u < low_pct / 100.0
    hi = (u >= low_pct / 100.0) & (u < (low_pct + high_pct) / 100.0)
    s[lo] = 0xDC00 + rng.integers(0, 1024, size=int(lo.sum()))
    s[hi] = 0xD800 + rng.integers(0, 1024, size=int(hi.sum()))
    return s.astype(np.uint16)


PAPER_SWEEP_POINTS = 128


def paper_sweep_sizes(points=PAPER_SWEEP_POINTS, top=1_000_000) -> np.ndarray:
    """The size sweep of Sec. 4 (throughput from 0 to a million units): the
    sizes top * k / points for k = 1..points."""
    return (np.arange(1, points + 1, dtype=np.int64) * top) // points


def paper_sweep_string(i: int, sizes=None) -> np.ndarray:
    """A fresh string for sweep point i: the paper's generator at 0.1 %
    pairs and 0.1 % mismatched, seeded per point."""
    sizes = paper_sweep_sizes() if sizes is None else sizes
    return paper_mix(int(sizes[i]), 0.1, 0.1, [SEEDS["paper_sweep"], int(i)])


def paper_1m_batch(mis_pct: float, k=64):
    """(buf, offsets): k strings of 1,000,000 units from the paper's
    generator at 0.1 % pairs and mis_pct percent mismatched."""
    buf = paper_mix(1_000_000 * k, 0.1, mis_pct, SEEDS["paper_1m"] + 1)
    return buf, np.arange(0, 1_000_000 * (k + 1), 1_000_000, dtype=np.int64)


def js_batch(k=1 << 18, distinct=64, seed=SEEDS["js_1024"] + 1):
    """(buf, offsets): k JavaScript-shape strings of 1024 units, `distinct`
    freshly drawn ones repeated in turn (distinct = k draws them all)."""
    rng = _rng(seed)
    one = np.concatenate([js_string(seed=rng) for _ in range(distinct)])
    buf = np.tile(one, k // distinct) if k % distinct == 0 else np.resize(one, 1024 * k)
    return buf, np.arange(0, 1024 * (k + 1), 1024, dtype=np.int64)


def serve_schedule(duration_s: float, rate_hz=50_000.0, seed=SEEDS["serve"], max_len=1 << 24,
                   n_pools=16, pool_len=1 << 25, min_len=1):
    """Poisson arrival schedule for the serving loop.

    Returns a dict of numpy arrays, one entry per request: ``arrival_ns``
    (sorted), ``length`` (Zipf(1.1) over 1..max_len, capped to the pool
    length), ``rate`` (lone-surrogate rate, log-uniform over [1e-6, 1e-1]),
    ``pool`` (index of the pool whose rate is nearest in log space) and
    ``pool_offset`` (uniform start inside that pool), plus ``pool_rates``."""
    rng = _rng(seed)
    count = int(rng.poisson(rate_hz * duration_s))
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    arrival = np.cumsum(gaps)
    lens = np.minimum(zipf_lengths(count, rng, max_len=max_len), pool_len)
    lens = np.maximum(lens, min_len)
    rates = 10.0 ** rng.uniform(-6.0, -1.0, size=count)
    pool_rates = np.logspace(-6.0, -1.0, n_pools)
    pool = np.abs(np.log10(rates)[:, None] - np.log10(pool_rates)[None, :]).argmin(axis=1)
    offs = rng.integers(0, pool_len - lens + 1)
    return {
        "arrival_ns": (arrival * 1e9).astype(np.int64),
        "length": lens.astype(np.int64),
        "rate": rates,
        "pool": pool.astype(np.int32),
        "pool_offset": offs.astype(np.int64),
        "pool_rates": pool_rates,
    }


def serve_pools(pool_rates, pool_len=1 << 25, seed=SEEDS["serve"] + 1):
    """One mix(r_j) pool of ``pool_len`` units per rate r_j."""
    rng = _rng(seed)
    return [mix(pool_len, float(r), rng) for r in pool_rates]
