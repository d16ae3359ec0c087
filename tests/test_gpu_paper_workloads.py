"""The paper's own workloads on the GPU, launched as the benchmark launches
them (the device's tuning cache applied, the same size hints), bit-exact
against the oracle: the two fixed 1,000,000-unit runs at 0.1 % pairs with
0 % and 0.1 % mismatched and the 128-point size sweep (Sec. 4), and the
1024-unit JavaScript string with 5 % lone lows and 5 % lone highs (Sec. 4.1).
Each flat, as a batch in one launch, and served."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2601_06349_amd import workloads as W
from tests.gpu_util import assert_same, log, offsets_dev, to_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu

SENTINEL = 0x1234


@pytest.fixture(scope="module")
def wf():
    torch_mod()
    import paper_2601_06349_amd as wf
    from paper_2601_06349_amd import tune
    wf.reset_params()
    name = tune.apply_cache()
    assert name is not None, "no tuning cache for this device: the benchmark's shapes cannot be reproduced"
    log(f"tuning cache {name}")
    yield wf
    wf.reset_params()


def _flat(wf, s, phase_in, phase_out, what):
    """Out of place, in place, isWellFormed and locate of one string against
    the oracle; nothing outside the output is written."""
    want, cnt = oracle.to_well_formed_count(s)
    t_in, _ = to_dev(s, phase_in, pad=8)
    t_out, base_out = to_dev(np.full(s.size, SENTINEL, np.uint16), phase_out, pad=8)
    wf.utf16_to_well_formed(t_in, t_out)
    assert_same(to_host(t_out), want, f"{what}: repair, phases {phase_in}/{phase_out}")
    host = to_host(base_out)
    start = phase_out + 8
    assert np.all(host[:start] == SENTINEL) and np.all(host[start + s.size:] == SENTINEL), what
    t_ip, _ = to_dev(s, phase_in, pad=8)
    wf.utf16_to_well_formed_inplace(t_ip)
    assert_same(to_host(t_ip), want, f"{what}: in place, phase {phase_in}")
    assert wf.is_well_formed(t_in) == (cnt == 0), f"{what}: isWellFormed"
    loc = wf.utf16_locate_ill_formed(t_in).cpu().numpy()
    assert int(loc[0]) == oracle.first_bad(s) and int(loc[1]) == cnt, f"{what}: locate"


def _batch(wf, buf, off, what, hint):
    """Every batch operation through the general entry with the given size
    hint (the benchmark's call), against the oracle per string."""
    torch = torch_mod()
    b = off.size - 1
    want = oracle.to_well_formed_batch(buf, off)
    t_in = torch.from_numpy(buf.view(np.int16)).cuda()
    t_off = offsets_dev(off)
    t_out = torch.full_like(t_in, SENTINEL)
    log(f"{what}: {b} strings, {buf.size} units, hint {hint}")
    wf.utf16wf_batch(wf.OP_TO, t_in, t_off, out=t_out, units_hint=hint)
    assert_same(to_host(t_out), want, f"{what}: batch repair")
    t_ip = t_in.clone()
    wf.utf16wf_batch(wf.OP_TO_INPLACE, t_ip, t_off, out=t_ip, units_hint=hint)
    assert_same(to_host(t_ip), want, f"{what}: batch repair in place")
    del t_ip, t_out
    res = torch.empty(b, dtype=torch.uint8, device="cuda")
    wf.utf16wf_batch(wf.OP_IS, t_in, t_off, results=res, units_hint=hint)
    assert np.array_equal(res.cpu().numpy(), oracle.is_well_formed_batch(buf, off)), f"{what}: batch check"
    first = torch.empty(b, dtype=torch.int64, device="cuda")
    count = torch.empty(b, dtype=torch.int64, device="cuda")
    wf.utf16wf_batch(wf.OP_LOCATE, t_in, t_off, first=first, count=count, units_hint=hint)
    wf_first, wf_count = oracle.locate_batch(buf, off)
    assert np.array_equal(first.cpu().numpy(), wf_first), f"{what}: batch locate, first"
    assert np.array_equal(count.cpu().numpy(), wf_count), f"{what}: batch locate, count"
    del t_in
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mis", [0.0, 0.1])
def test_paper_1m_runs_flat(wf, mis):
    s = W.paper_mix(1_000_000, 0.1, mis, W.SEEDS["paper_1m"])
    for pi, po in ((0, 0), (3, 3), (5, 1)):
        log(f"paper 1M mis={mis}: phases {pi}/{po}")
        _flat(wf, s, pi, po, f"1M, {mis} % mismatched")


@pytest.mark.parametrize("mis", [0.0, 0.1])
def test_paper_1m_runs_batch_of_64(wf, mis):
    buf, off = W.paper_1m_batch(mis)
    _batch(wf, buf, off, f"64 x 1M, {mis} % mismatched", hint=buf.size)


def test_size_sweep_fresh_strings(wf):
    """All 128 sweep points, each a fresh string, at input phase 0 and at a
    non-zero phase (with an equal and with a different output phase), then
    all 128 as one batch."""
    sizes = W.paper_sweep_sizes()
    strings = []
    for i in range(sizes.size):
        s = W.paper_sweep_string(i, sizes)
        strings.append(s)
        log(f"sweep point {i}: {s.size} units")
        _flat(wf, s, 0, 0, f"sweep {s.size}")
        _flat(wf, s, 3, 3 if i % 2 else 6, f"sweep {s.size}")
    buf = np.concatenate(strings)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    _batch(wf, buf, off, "the 128 sweep strings", hint=buf.size)


def test_js_1024_flat(wf):
    s = W.js_string()
    for phase in range(8):
        _flat(wf, s, phase, (phase * 3) % 8, "JS 1024")


def test_js_1024_batch_as_benchmarked(wf):
    buf, off = W.js_batch()
    _batch(wf, buf, off, "262,144 JS strings (64 distinct)", hint=buf.size)


def test_js_1024_batch_all_distinct(wf):
    # every unit drawn independently: 262,144 independent 1024-unit strings
    k = 1 << 18
    buf = W.js_string(n=1024 * k, seed=W.SEEDS["js_1024"] + 2)
    off = np.arange(0, 1024 * (k + 1), 1024, dtype=np.int64)
    _batch(wf, buf, off, "262,144 distinct JS strings", hint=buf.size)


def _check_served(torch, summ, dst, pool, which, length, what):
    assert summ["all_completed"] and summ["completed"] == which.size, f"{what}: {summ}"
    want = oracle.to_well_formed_batch(pool, np.arange(0, pool.size + 1, length, dtype=np.int64))
    got = to_host(dst)[:which.size * length].reshape(which.size, length)
    want = want.reshape(-1, length)
    bad = np.nonzero(np.any(got != want[which], axis=1))[0]
    assert bad.size == 0, f"{what}: {bad.size} of {which.size} requests differ, first {bad[:5]}"


def test_js_1024_served(wf):
    """1,000,000 requests/s of 1024-unit strings for one second (the
    benchmark's run), each into a destination of its own: every output
    equals the oracle's."""
    torch = torch_mod()
    from paper_2601_06349_amd import serve as S
    pool, arrival, which = S.js_requests()
    dst = torch.full((which.size * 1024,), SENTINEL, dtype=torch.int16, device="cuda")
    summ = S.serve_js_strings(dst=dst, log=log)
    log(f"served: p50 {summ.get('p50_ms')} ms, p99 {summ.get('p99_ms')} ms, {summ['stats']}")
    _check_served(torch, summ, dst, pool, which, 1024, "served JS strings")
    del dst
    torch.cuda.empty_cache()


def test_paper_1m_runs_served(wf):
    """The two 1,000,000-unit runs as requests at 10,000/s for 0.1 s, each
    into a destination of its own: every output equals the oracle's."""
    torch = torch_mod()
    from paper_2601_06349_amd import serve as S
    pool, arrival, which = S.paper_1m_requests()
    dst = torch.full((which.size * 1_000_000,), SENTINEL, dtype=torch.int16, device="cuda")
    summ = S.serve_paper_1m(dst=dst, log=log)
    log(f"served: p50 {summ.get('p50_ms')} ms, p99 {summ.get('p99_ms')} ms, {summ['stats']}")
    _check_served(torch, summ, dst, pool, which, 1_000_000, "served 1M runs")
    del dst
    torch.cuda.empty_cache()
