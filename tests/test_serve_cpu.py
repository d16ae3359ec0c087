"""The serving loop's scheduler on a simulated device (virtual clock, no
GPU): admission under the HBM budget, arrival order, continuous batching,
concurrency limit, time-outs, launch-failure handling."""
from __future__ import annotations

import numpy as np
import pytest

import paper_2601_06349_amd as wf
from paper_2601_06349_amd import serve as S


def _layout_bytes(nreq, units):
    r = lambda b: (b + 255) // 256 * 256
    return r(2 * units) + r(2 * units + 16 * nreq) + r(max(nreq, 1))


def test_budget_and_rejection():
    rng = np.random.default_rng(0)
    n = 400
    arr = np.sort(rng.integers(0, 2_000_000, size=n))
    lens = rng.integers(0, 20_000, size=n)
    lens[[5, 77]] = 1_000_000  # larger than the whole arena
    arena = 200_000
    cfg = S.make_config(num_streams=3, arena_bytes=arena, max_batch_requests=16, max_batch_units=50_000)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=5_000, lat_ns_per_unit=2.0)
    assert st["arena_peak_bytes"] <= arena
    assert list(np.nonzero(out["status"] == wf.ERANGE)[0]) == [5, 77]
    assert st["rejected"] == 2 and st["completed"] == n - 2
    assert np.all(out["status"][out["status"] != wf.ERANGE] == 0)
    # every batch fits the arena and respects the limits
    for b in np.unique(out["batch"][out["batch"] >= 0]):
        m = out["batch"] == b
        assert m.sum() <= 16
        assert lens[m].sum() <= 50_000 or m.sum() == 1
        assert _layout_bytes(int(m.sum()), int(lens[m].sum())) <= arena
    assert st["max_inflight"] <= 3


def test_arrival_order_and_no_early_launch():
    rng = np.random.default_rng(1)
    n = 1000
    arr = np.cumsum(rng.exponential(2_000, size=n)).astype(np.int64)
    lens = rng.integers(1, 5_000, size=n)
    cfg = S.make_config(num_streams=4, arena_bytes=1 << 30, max_batch_requests=64, max_batch_units=100_000)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=30_000, lat_ns_per_unit=1.0)
    assert np.all(out["status"] == 0)
    assert np.all(out["launch_ns"] >= arr)
    assert np.all(out["done_ns"] > out["launch_ns"])
    # admitted in arrival order: batch ids never decrease along the arrivals
    assert np.all(np.diff(out["batch"]) >= 0)


def test_continuous_batching_fills_next_batch():
    """One slot, 100 us per batch, a request every 10 us: the first batch holds
    one request and each later batch holds every request that arrived while
    the previous one was on the device."""
    n = 50
    arr = np.arange(n, dtype=np.int64) * 10_000
    lens = np.full(n, 100)
    cfg = S.make_config(num_streams=1, arena_bytes=1 << 30, max_batch_requests=1000, max_batch_units=1 << 30)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=100_000, lat_ns_per_unit=0.0)
    assert out["batch"][0] == 0 and np.sum(out["batch"] == 0) == 1
    sizes = np.bincount(out["batch"])
    assert np.all(sizes[1:-1] == 10), sizes
    for b in range(1, sizes.size):
        m = out["batch"] == b
        t = out["launch_ns"][m][0]
        waiting = (arr <= t) & (out["batch"] >= b)
        assert np.array_equal(np.nonzero(waiting)[0], np.nonzero(m)[0])


def test_overlap_uses_all_slots():
    n = 200
    arr = np.zeros(n, dtype=np.int64)
    lens = np.full(n, 1000)
    cfg = S.make_config(num_streams=4, arena_bytes=1 << 30, max_batch_requests=5, max_batch_units=1 << 30)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=50_000)
    assert st["max_inflight"] == 4
    assert st["batches"] == 40
    assert len(np.unique(out["slot"])) == 4


def test_memory_blocks_admission_until_free():
    """Two requests that each need most of the arena run one after the other
    even with free slots."""
    arena = _layout_bytes(1, 30_000) + 500
    arr = np.zeros(3, dtype=np.int64)
    lens = np.array([30_000, 30_000, 10])
    cfg = S.make_config(num_streams=4, arena_bytes=arena, max_batch_requests=1, max_batch_units=1 << 30)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=10_000)
    assert out["launch_ns"][1] >= out["done_ns"][0]
    assert out["launch_ns"][2] >= out["launch_ns"][1]  # arrival order is kept
    assert st["max_inflight"] == 1


def test_timeouts():
    n = 100
    arr = np.zeros(n, dtype=np.int64)
    lens = np.full(n, 10)
    cfg = S.make_config(num_streams=1, arena_bytes=1 << 30, max_batch_requests=1, max_batch_units=1 << 30,
                        timeout_ns=250_000)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=100_000)
    assert st["timed_out"] > 0 and st["completed"] + st["timed_out"] == n
    assert np.all(out["status"][:3] == 0)
    assert np.all((out["status"] == 0) | (out["status"] == 1))


def test_launch_failures_are_reported_and_loop_continues():
    n = 60
    arr = np.arange(n, dtype=np.int64) * 1000
    lens = np.full(n, 10)
    cfg = S.make_config(num_streams=2, arena_bytes=1 << 30, max_batch_requests=1, max_batch_units=1 << 30)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=5_000, fail_every=3)
    assert st["failed"] == 20 and st["completed"] == 40
    assert np.all(out["status"][2::3] == wf.EHIP)
    assert st["arena_peak_bytes"] > 0


def test_deterministic_and_edge_cases():
    rng = np.random.default_rng(5)
    arr = np.sort(rng.integers(0, 10_000_000, size=300))
    lens = rng.integers(0, 3, size=300)  # many empty requests
    cfg = S.make_config(num_streams=2, arena_bytes=1 << 20, max_batch_requests=7, max_batch_units=1000)
    a, sa = S.simulate(arr, lens, cfg)
    b, sb = S.simulate(arr, lens, cfg)
    assert np.array_equal(a, b) and sa == sb
    assert np.all(a["status"] == 0)
    out, st = S.simulate(np.zeros(0, np.int64), np.zeros(0, np.int64), cfg)
    assert st["batches"] == 0


def test_argument_errors():
    cfg = S.make_config(num_streams=0)
    with pytest.raises(wf.Utf16wfError):
        S.simulate([0], [1], cfg)
    cfg = S.make_config(num_streams=2)
    with pytest.raises(wf.Utf16wfError):
        S.simulate([5, 3], [1, 1], cfg)
    with pytest.raises(wf.Utf16wfError):
        S.simulate([0], [-1], cfg)
    cfg = S.make_config(num_streams=2, op=wf.OP_LOCATE)
    with pytest.raises(wf.Utf16wfError):
        S.simulate([0], [1], cfg)
    for bad in (-2, 33):
        with pytest.raises(wf.Utf16wfError):
            S.simulate([0], [1], S.make_config(num_streams=2, separate_max=bad))


def test_run_rejects_bad_requests_before_any_device_call():
    """utf16wf_serve_run checks every request before touching the device, so
    these run without a GPU: fake, never dereferenced device addresses."""
    A = 0x100000
    cfg = S.make_config(num_streams=2, arena_bytes=1 << 20)

    def reqs(*rows):
        r = np.zeros(len(rows), dtype=S.REQUEST_DTYPE)
        for i, (t, src, n, dst) in enumerate(rows):
            r[i] = (t, src, n, dst)
        return r

    cases = [
        (reqs((0, A, 10, A + 10)), wf.EOVERLAP),         # destination overlaps its payload
        (reqs((0, A + 10, 10, A)), wf.EOVERLAP),
        (reqs((0, A + 1, 10, 0)), wf.EALIGN),            # odd payload address
        (reqs((0, A, 10, A + 4097)), wf.EALIGN),         # odd destination
        (reqs((0, 0, 10, 0)), wf.EINVAL),                # null payload
        (reqs((0, A, -1, 0)), wf.EINVAL),                # negative length
        (reqs((5, A, 1, 0), (4, A, 1, 0)), wf.EINVAL),   # decreasing arrivals
    ]
    for r, code in cases:
        with pytest.raises(wf.Utf16wfError) as e:
            S.run(r, cfg)
        assert e.value.code == code, (r, e.value)
    with pytest.raises(wf.Utf16wfError):
        S.run(reqs((0, A, 1, 0)), S.make_config(num_streams=17))


def test_latency_summary():
    arr = np.arange(10, dtype=np.int64) * 1_000_000
    lens = np.full(10, 1000)
    cfg = S.make_config(num_streams=1)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=500_000)
    s = S.latency_summary(out, arr, lens)
    assert s["completed"] == 10 and abs(s["p50_ms"] - 0.5) < 1e-6 and abs(s["p99_ms"] - 0.5) < 1e-6
    assert 0.0 < s["inflight_frac"] <= 1.0


def test_failed_launch_region_held_until_its_queued_work_drains():
    """A launch that fails after part of its batch was queued (a copy, the
    gather) must not hand its arena region to the next batch before that
    work is done: the simulator queues a failing batch's work first and
    reports any launch whose region such work could still write."""
    n = 40
    arr = np.zeros(n, dtype=np.int64)
    lens = np.full(n, 20_000)
    arena = 2 * _layout_bytes(1, 20_000)  # room for two batches: regions are reused at once
    lat = 50_000
    cfg = S.make_config(num_streams=2, arena_bytes=arena, max_batch_requests=1, max_batch_units=1 << 30)
    out, st = S.simulate(arr, lens, cfg, lat_base_ns=lat, lat_ns_per_unit=0.0, fail_every=2)
    assert st["failed"] == n // 2 and st["completed"] == n // 2
    failed = np.nonzero(out["status"] == wf.EHIP)[0]
    assert np.array_equal(failed, np.arange(1, n, 2))
    # the batch after a failed one waits for the failed batch's queued work
    for i in failed[failed + 1 < n]:
        assert out["launch_ns"][i + 1] >= out["launch_ns"][i] + lat
    assert st["arena_peak_bytes"] <= arena


def test_slice_expectations_equal_the_oracle_on_each_slice():
    """The full serving test's expected outputs (the oracle over each pool,
    with a slice's two end units from the oracle over those units alone)
    equal the oracle run on each slice by itself."""
    import oracle
    from tests.test_gpu_serve import _slice_expectations
    rng = np.random.default_rng(12)
    pool_len = 4096
    alphabet = np.array([0x41, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0x4E2D], np.uint16)
    pools_all = alphabet[rng.integers(0, alphabet.size, size=3 * pool_len)]
    want_all = oracle.to_well_formed_batch(pools_all, np.arange(0, pools_all.size + 1, pool_len, dtype=np.int64))
    k = 3000
    p = rng.integers(0, 3, size=k)
    lens = rng.integers(1, 40, size=k)
    lens[:5] = [1, 2, 3, pool_len, pool_len - 1]
    o = np.array([rng.integers(0, pool_len - ln + 1) for ln in lens])
    o[3] = 0
    g = p * pool_len + o
    first, last = _slice_expectations(pools_all, g, lens)
    for i in range(k):
        want = want_all[g[i]:g[i] + lens[i]].copy()
        want[0], want[-1] = first[i], last[i]
        assert np.array_equal(want, oracle.to_well_formed(pools_all[g[i]:g[i] + lens[i]])), i
