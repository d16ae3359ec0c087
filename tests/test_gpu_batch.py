"""GPU parity of the ragged-batch entry points and batch plans against the
CPU oracle (per-string repair), bit-exact."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from paper_2601_06349_amd import workloads as W
from tests.gpu_util import assert_same, log, offsets_dev, to_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu

H, L, A = 0xD801, 0xDC02, 0x0041
ROWS = (1, 2, 4, 8)


@pytest.fixture(scope="module")
def wf():
    torch_mod()
    import paper_2601_06349_amd as wf
    wf.reset_params()
    yield wf
    wf.reset_params()


def _force_rows(wf, rows, wg_waves=4, grid_per_cu=8, nt=0, store_lines=1):
    for op in (wf.OP_IS, wf.OP_TO, wf.OP_TO_INPLACE, wf.OP_LOCATE):
        wf.set_params(op, 1, -1, rows=rows, wg_waves=wg_waves, grid_per_cu=grid_per_cu, nontemporal=nt,
                      store_lines=store_lines)
    # (a locate over few strings takes the flat parameters)
    wf.set_params(wf.OP_LOCATE, 0, -1, rows=rows, wg_waves=wg_waves, grid_per_cu=grid_per_cu, nontemporal=nt)


def _check_batch(wf, buf, off, phase_in=0, phase_out=0, what="", hint=0):
    torch = torch_mod()
    off = np.asarray(off, np.int64)
    b = off.size - 1
    sentinel = np.full(buf.size, 0x1234, np.uint16)
    want = oracle.to_well_formed_batch(buf, off, out=sentinel)
    want_ip = oracle.to_well_formed_batch(buf, off)
    t_in, _ = to_dev(buf, phase_in, pad=8)
    t_off = offsets_dev(off)
    t_out, _ = to_dev(sentinel, phase_out, pad=8)
    if hint:
        wf.utf16wf_batch(wf.OP_TO, t_in, t_off, out=t_out, units_hint=hint)
    else:
        wf.utf16_to_well_formed_batch(t_in, t_off, out=t_out)
    assert_same(to_host(t_out), want, f"batch oop {what} phase {phase_in}/{phase_out}")
    t_ip, _ = to_dev(buf, phase_in, pad=8)
    wf.utf16_to_well_formed_batch_inplace(t_ip, t_off)
    assert_same(to_host(t_ip), want_ip, f"batch inplace {what}")
    if hint:
        res_t = torch.empty(b, dtype=torch.uint8, device="cuda")
        wf.utf16wf_batch(wf.OP_IS, t_in, t_off, results=res_t, units_hint=hint)
        res = res_t.cpu().numpy()
    else:
        res = wf.utf16_is_well_formed_batch(t_in, t_off).cpu().numpy()
    want_res = oracle.is_well_formed_batch(buf, off)
    assert np.array_equal(res, want_res), f"batch is {what}: {np.nonzero(res != want_res)[0][:10]}"
    if hint:
        first = torch.empty(b, dtype=torch.int64, device="cuda")
        cnt = torch.empty(b, dtype=torch.int64, device="cuda")
        wf.utf16wf_batch(wf.OP_LOCATE, t_in, t_off, first=first, count=cnt, units_hint=hint)
    else:
        first, cnt = wf.utf16_locate_ill_formed_batch(t_in, t_off)
    wf_first, wf_cnt = oracle.locate_batch(buf, off)
    assert np.array_equal(first.cpu().numpy(), wf_first), f"batch first_bad {what}"
    assert np.array_equal(cnt.cpu().numpy(), wf_cnt), f"batch count {what}"
    torch.cuda.synchronize()
    return b


def _random_batch(rng, b, max_len, alphabet, pre=0, post=0):
    lens = rng.integers(0, max_len + 1, size=b)
    if int(lens.sum()) + pre + post == 0:
        post = 1  # keep the buffer non-empty so it has a device address
    total = int(lens.sum()) + pre + post
    buf = alphabet[rng.integers(0, alphabet.size, size=total)].astype(np.uint16)
    off = np.concatenate([[pre], pre + np.cumsum(lens)]).astype(np.int64)
    return buf, off


@pytest.mark.parametrize("rows", ROWS)
def test_random_batches(wf, rows):
    _force_rows(wf, rows)
    rng = np.random.default_rng(rows)
    alphabet = np.array([A, 0x4E2D, H, L, 0xDBFF, 0xDFFF], np.uint16)
    for i, (b, max_len) in enumerate([(1, 0), (1, 1), (3, 5), (40, 12), (300, 40), (1000, 3), (50, 3000),
                                      (7, 9000)]):
        buf, off = _random_batch(rng, b, max_len, alphabet, pre=i % 5, post=(3 * i) % 7)
        _check_batch(wf, buf, off, what=f"rows={rows} b={b} max={max_len}")
    wf.reset_params()


def test_phases(wf):
    rng = np.random.default_rng(42)
    alphabet = np.array([A, H, L], np.uint16)
    buf, off = _random_batch(rng, 500, 30, alphabet, pre=3, post=2)
    for pi, po in itertools.product((0, 3, 7), range(8)):  # every relative output phase
        _check_batch(wf, buf, off, pi, po, what="phases")


def test_no_pairing_across_strings(wf):
    """Every string ends in a high and the next starts with a low: a flat
    repair of the concatenation would keep these pairs; the batch must not."""
    rng = np.random.default_rng(1)
    lens = rng.integers(2, 20, size=5000)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    buf = np.full(int(off[-1]), A, np.uint16)
    buf[off[1:] - 1] = H
    buf[off[:-1]] = L
    flat = oracle.to_well_formed(buf)
    per = oracle.to_well_formed_batch(buf, off)
    assert not np.array_equal(flat, per)
    _check_batch(wf, buf, off, what="adversarial ends")


def test_tiny_and_empty_strings(wf):
    """Thousands of one-unit strings per tile and long runs of empty strings
    at one position (more than a wave's worth of offsets per scan step)."""
    for rows in ROWS:
        _force_rows(wf, rows)
        buf = np.tile(np.array([H, L, A, L, H], np.uint16), 3000)
        off = np.arange(buf.size + 1, dtype=np.int64)
        _check_batch(wf, buf, off, what=f"unit strings rows={rows}")
        lens = np.zeros(700, np.int64)
        lens[::100] = 37
        lens[350] = 5000
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        buf = W.mix(int(off[-1]), 0.05, 9)
        _check_batch(wf, buf, off, what=f"empty runs rows={rows}")
        off = np.zeros(300, np.int64)  # all strings empty
        _check_batch(wf, np.zeros(10, np.uint16) + H, off, what="all empty")
    wf.reset_params()


def test_offsets_per_tile_around_one_wave(wf):
    """Tiles holding 1, 2, 62, 63, 64, 65 and 200 offsets, with repeats
    (empty strings) and dense surrogates: around 64 offsets per tile the
    check and the locate switch between the tile's offsets kept in the wave's
    lanes and a search in memory; both must name the same strings."""
    rng = np.random.default_rng(11)
    alphabet = np.array([A, H, L, 0xDBFF, 0xDC00, A], np.uint16)
    for rows in ROWS:
        _force_rows(wf, rows)
        t = 512 * rows
        starts = [0]
        counts = [1, 2, 62, 63, 64, 65, 200] * 3
        for i, c in enumerate(counts):
            tl = (i + 1) * t  # tile 0 holds only the first string's start
            pos = np.sort(rng.integers(tl, tl + t, size=c))
            if i % 3 == 0:
                pos[0] = tl  # a start exactly on the tile's first unit
            starts.extend(pos.tolist())
        total = (len(counts) + 1) * t + 37
        off = np.array(starts + [total], np.int64)
        buf = alphabet[rng.integers(0, alphabet.size, size=total)].astype(np.uint16)
        _check_batch(wf, buf, off, what=f"offsets per tile rows={rows}")
    wf.reset_params()


@pytest.mark.parametrize("nstr", (65536, 65537))
def test_many_short_strings_at_the_search_switch(wf, nstr):
    """65,536 strings (the check scans each tile's offsets before its loads
    and skips strings already known bad) and 65,537 (it loads first), short
    strings with empty ones, a few long ones, dense surrogates."""
    rng = np.random.default_rng(nstr)
    lens = rng.integers(0, 40, size=nstr)
    lens[rng.integers(0, nstr, size=20)] = rng.integers(5000, 20000, size=20)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    buf = W.mix(int(off[-1]), 0.002, 77)
    for k in rng.integers(0, nstr, size=500):  # lone surrogates at string edges
        if lens[k]:
            buf[off[k]] = L
            buf[off[k + 1] - 1] = H
    _check_batch(wf, buf, off, what=f"nstr={nstr}")
    _check_batch(wf, buf, off, what=f"nstr={nstr} hinted", hint=int(off[-1]))


def test_long_string_among_short(wf):
    rng = np.random.default_rng(5)
    lens = rng.integers(1, 50, size=2000)
    lens[1000] = 3_000_017
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    buf = W.mix(int(off[-1]), 1e-3, 6)
    _check_batch(wf, buf, off, what="long among short")
    _check_batch(wf, buf, off, what="long among short, hinted", hint=int(off[-1]))


def test_is_early_exit_long_bad_strings(wf):
    """Long ill-formed strings whose later tiles are skipped once the first
    error is known; every result must still be exact."""
    lens = np.array([2_000_000, 5, 1_500_000, 1, 3_000_000], np.int64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    buf = W.ascii_units(int(off[-1]), 3)
    buf[10] = H  # string 0 bad at its start
    buf[off[2] + 1_400_000] = L  # string 2 bad near its end
    buf[off[4]] = L
    for rows in ROWS:
        _force_rows(wf, rows)
        _check_batch(wf, buf, off, what=f"early exit rows={rows}")
    wf.reset_params()


def test_plans_replay(wf):
    torch = torch_mod()
    rng = np.random.default_rng(11)
    buf, off = _random_batch(rng, 3000, 25, np.array([A, H, L], np.uint16))
    t_in, _ = to_dev(buf)
    t_off = offsets_dev(off)
    t_out, _ = to_dev(np.zeros_like(buf))
    res = torch.empty(off.size - 1, dtype=torch.uint8, device="cuda")
    p_to = wf.BatchPlan(wf.OP_TO, t_in, t_off, out=t_out)
    p_is = wf.BatchPlan(wf.OP_IS, t_in, t_off, results=res)
    for rep in range(4):
        cur = buf.copy()
        cur[rng.integers(0, buf.size, size=50)] = H  # new content each replay
        t_in.copy_(torch.from_numpy(cur.view(np.int16)))
        t_out.zero_()
        res.fill_(7)
        p_to.launch()
        p_is.launch()
        torch.cuda.synchronize()
        assert_same(to_host(t_out), oracle.to_well_formed_batch(cur, off), f"plan replay {rep}")
        assert np.array_equal(res.cpu().numpy(), oracle.is_well_formed_batch(cur, off)), f"plan is {rep}"
    # new boundaries (same number of strings, a different span): the shape
    # picked at creation no longer fits, the results must still be exact
    off2 = np.sort(rng.integers(0, buf.size + 1, size=off.size)).astype(np.int64)
    off2[0] = 5
    off2 = np.maximum(off2, 5)
    t_off.copy_(torch.from_numpy(off2))
    t_out.zero_()
    res.fill_(7)
    p_to.launch()
    p_is.launch()
    torch.cuda.synchronize()
    want = oracle.to_well_formed_batch(cur, off2, out=np.zeros_like(cur))
    assert_same(to_host(t_out), want, "plan replay, new offsets")
    assert np.array_equal(res.cpu().numpy(), oracle.is_well_formed_batch(cur, off2)), "plan is, new offsets"
    p_to.close()
    p_is.close()
    t_off.copy_(torch.from_numpy(off))
    # in-place plan
    t_ip, _ = to_dev(buf)
    p_ip = wf.BatchPlan(wf.OP_TO_INPLACE, t_ip, t_off)
    p_ip.launch()
    p_ip.launch()  # idempotent
    torch.cuda.synchronize()
    assert_same(to_host(t_ip), oracle.to_well_formed_batch(buf, off), "plan inplace")
    p_ip.close()


def test_results_at_any_alignment(wf):
    """Per-string results written into a byte buffer at odd offsets: the
    initialisation fills exactly the strings' bytes, head and tail included."""
    torch = torch_mod()
    rng = np.random.default_rng(21)
    for b in (1, 15, 16, 17, 3001):
        buf, off = _random_batch(rng, b, 30, np.array([A, H, L], np.uint16))
        t_in, _ = to_dev(buf)
        t_off = offsets_dev(off)
        want = oracle.is_well_formed_batch(buf, off)
        for shift in (0, 1, 3, 7, 13):
            for hint in (0, int(off[-1])):  # head pass sets the results / fill kernel does
                big = torch.full((b + 40,), 0x5A, dtype=torch.uint8, device="cuda")
                wf.utf16wf_batch(wf.OP_IS, t_in, t_off, results=big[shift:shift + b], units_hint=hint)
                got = big.cpu().numpy()
                assert np.array_equal(got[shift:shift + b], want), (b, shift, hint)
                assert np.all(got[:shift] == 0x5A) and np.all(got[shift + b:] == 0x5A), (b, shift, hint)


def test_validate_offsets(wf):
    good = offsets_dev(np.array([0, 3, 3, 10], np.int64))
    wf.utf16wf_validate_offsets(good, 10)
    for bad, n in (([0, 3, 2, 10], 10), ([0, 3, 5, 11], 10), ([-1, 3, 5, 9], 10)):
        with pytest.raises(wf.Utf16wfError) as e:
            wf.utf16wf_validate_offsets(offsets_dev(np.array(bad, np.int64)), n)
        assert e.value.code == wf.EOFFSETS


def test_ragged_1m_full(wf):
    """1,000,000 log-normal strings (about 98.6M units), with the tuned
    launch shapes the benchmark uses, launched with and without a size hint."""
    from paper_2601_06349_amd import tune
    tune.apply_cache()
    log("generating ragged_1m")
    buf, off = W.ragged_batch()
    log(f"ragged_1m: {off.size - 1} strings, {off[-1]} units")
    _check_batch(wf, buf, off, what="ragged_1m")
    _check_batch(wf, buf, off, what="ragged_1m hinted", hint=int(off[-1]))
    wf.reset_params()


def test_zipf_4096_full(wf):
    """4096 Zipf(1.1) strings up to 2^24 units (about 1.6G units), default
    shape: out of place, in place, is (early exit), locate."""
    torch = torch_mod()
    from paper_2601_06349_amd import tune
    tune.apply_cache()
    log("generating zipf_4096")
    buf, off, kind = W.zipf_batch()
    log(f"zipf_4096: {off[-1]} units, {int(kind.sum())} error strings")
    t_in = torch.from_numpy(buf.view(np.int16)).to("cuda")
    t_off = offsets_dev(off)
    want = oracle.to_well_formed_batch(buf, off)
    out = wf.utf16_to_well_formed_batch(t_in, t_off, out=torch.empty_like(t_in))
    assert_same(to_host(out), want, "zipf oop")
    del out
    res = wf.utf16_is_well_formed_batch(t_in, t_off).cpu().numpy()
    assert np.array_equal(res, oracle.is_well_formed_batch(buf, off))
    first, cnt = wf.utf16_locate_ill_formed_batch(t_in, t_off)
    of, oc = oracle.locate_batch(buf, off)
    assert np.array_equal(first.cpu().numpy(), of) and np.array_equal(cnt.cpu().numpy(), oc)
    wf.utf16_to_well_formed_batch_inplace(t_in, t_off)
    assert_same(to_host(t_in), want, "zipf inplace")
    del t_in
    torch.cuda.empty_cache()
    wf.reset_params()


def test_batch_beyond_32bit_indices(wf):
    """A batch over 2^31 + 2^21 + 5 units (4.3 GB): a string longer than 2^31
    units, 100,001 short strings past unit 2^31 (so the many-strings path
    runs on 64-bit offsets), mismatches planted inside them and across their
    boundaries. Repair, check and locate are checked on windows against the
    oracle and on every string's result; the same long string also goes
    through the serving loop as one request (the separate-strings kernel)."""
    torch = torch_mod()
    from paper_2601_06349_amd import serve as S
    G = 1 << 31
    n = G + (1 << 21) + 5
    small0 = G + 3000
    off = np.concatenate([[0, 1000], small0 + 10 * np.arange(100_002), [n]]).astype(np.int64)
    # string 1 = [1000, G + 3000): longer than 2^31 units
    plants = {G + 1500: [L], 500: [H], small0 + 10 * 7 + 9: [H], small0 + 10 * 8: [L],  # cut pair
              small0 + 10 * 500 + 4: [H, L], small0 + 10 * 900 + 4: [L, L], n - 1: [H]}
    t = torch.full((n,), A, dtype=torch.int16, device="cuda")
    for p, pat in plants.items():
        t[p:p + len(pat)] = torch.tensor(np.array(pat, np.uint16).view(np.int16), device="cuda")
    t_off = offsets_dev(off)
    out = torch.full_like(t, 0x1234)
    wf.utf16wf_batch(wf.OP_TO, t, t_off, out=out, units_hint=n)
    b = off.size - 1
    res = torch.empty(b, dtype=torch.uint8, device="cuda")
    wf.utf16wf_batch(wf.OP_IS, t, t_off, results=res, units_hint=n)
    first, count = wf.utf16_locate_ill_formed_batch(t, t_off)
    res, first, count = res.cpu().numpy(), first.cpu().numpy(), count.cpu().numpy()
    bad = set()
    for p in plants:
        a0, b0 = max(0, p - 40), min(n, p + 40)
        win = to_host(t[a0:b0])
        # the strings inside the window, clipped to it
        ks = np.searchsorted(off, [a0, b0], side="right") - 1
        cuts = np.unique(np.clip(off[max(ks[0], 0):min(ks[1] + 2, off.size)], a0, b0)) - a0
        cuts = np.concatenate([[0], cuts[(cuts > 0) & (cuts < b0 - a0)], [b0 - a0]]).astype(np.int64)
        w = oracle.to_well_formed_batch(win, cuts)
        # a window end inside the buffer cuts a unit from its neighbour:
        # compare the units that keep both
        i0, i1 = (1 if a0 > 0 else 0), (b0 - a0) - (1 if b0 < n else 0)
        assert_same(to_host(out[a0 + i0:a0 + i1]), w[i0:i1], f"repair window at {p}")
        bad.update(int(u) for u in a0 + i0 + np.nonzero(w[i0:i1] != win[i0:i1])[0])
    want_first = np.full(b, -1, np.int64)
    want_count = np.zeros(b, np.int64)
    for u in sorted(bad):
        k = int(np.searchsorted(off, u, side="right") - 1)
        want_count[k] += 1
        if want_first[k] < 0:
            want_first[k] = u - off[k]
    assert len(bad) == 7  # the H, L pair is valid
    assert np.array_equal(count, want_count) and np.array_equal(first, want_first)
    assert np.array_equal(res, (want_count == 0).astype(np.uint8))
    assert first[1] == G + 500  # a first index past 2^31 inside its string
    # the long string as one served request (separate strings), into `out`
    out.fill_(0x1234)
    req = np.zeros(1, dtype=S.REQUEST_DTYPE)
    req["src"] = t.data_ptr() + 2 * 1000
    req["length"] = int(off[2] - off[1])
    req["dst"] = out.data_ptr() + 2 * 1000
    outc, st = S.run(req, S.make_config(num_streams=1, arena_bytes=12 << 30, max_batch_requests=1))
    assert outc["status"][0] == 0 and st["direct_batches"] == 1
    assert_same(to_host(out[G + 1492:G + 1508]), np.array([A] * 8 + [0xFFFD] + [A] * 7, np.uint16),
                "served window")
    assert_same(to_host(out[992:1008]), np.array([0x1234] * 8 + [A] * 8, np.uint16), "served start")
    end = int(off[2])
    assert_same(to_host(out[end - 8:end + 8]), np.array([A] * 8 + [0x1234] * 8, np.uint16), "served end")
    del t, out
    torch.cuda.empty_cache()


def test_head_check_boundaries(wf):
    """Batches of few long strings get a head check of each string's first
    512 units: a pair across unit 511/512 is valid, a lone high at 511 is not,
    strings just under and at the 8192-unit threshold, mismatches just past
    the head."""
    cases = []  # (length, {position: unit})
    cases.append((8192, {511: H, 512: L}))        # valid pair across the head edge
    cases.append((8192, {511: H}))                # lone high at the head's last unit
    cases.append((8191, {0: L}))                  # below the threshold: main pass only
    cases.append((8192, {0: L}))
    cases.append((10000, {512: L}))               # first mismatch just past the head
    cases.append((9000, {}))                      # well-formed
    cases.append((20000, {510: H, 511: L, 19999: H}))
    lens = np.array([c[0] for c in cases], np.int64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    buf = np.full(int(off[-1]), A, np.uint16)
    for k, (_, plants) in enumerate(cases):
        for p, u in plants.items():
            buf[off[k] + p] = u
    for hint in (0, int(off[-1])):
        _check_batch(wf, buf, off, what=f"head check hint={hint}", hint=hint)
    for phase in (1, 6):
        _check_batch(wf, buf, off, phase, phase, what=f"head check phase {phase}")


def test_check_results_every_clearing_path(wf):
    """Check results cleared by each kind of store: long strings with a clean
    head whose later tiles all hold errors (many waves find them at once and
    clear the result through their cache), a single error late in a long
    string (published device-wide by the wave that read a clean tile of it
    first), short strings ending inside a tile of several with an error at
    their end, and strings that go on past such a tile with an error in it.
    The same results buffer then serves a second batch in which those strings
    are well-formed: no cleared byte of the first call may show in the
    second."""
    torch = torch_mod()
    rng = np.random.default_rng(11)
    lens, kinds = [], []
    for rep in range(3):
        for n, kind in ((300_000, "dense"), (3, "end"), (250_000, "late"), (9000, "past_head"),
                        (200_000, "dense"), (40_000, "first_tile")):
            lens.append(n)
            kinds.append(kind)
        for _ in range(30):
            lens.append(int(rng.integers(1, 300)))
            kinds.append("end" if rng.random() < 0.5 else "clean")
    lens = np.array(lens, np.int64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    buf = W.ascii_units(int(off[-1]), 12)
    for k, kind in enumerate(kinds):
        s0, s1 = int(off[k]), int(off[k + 1])
        if kind == "dense":
            buf[s0 + 1000:s1:97] = L
        elif kind == "end":
            buf[s1 - 1] = H
        elif kind == "late":
            buf[s0 + (s1 - s0) * 4 // 5] = L
        elif kind == "past_head":
            buf[s0 + 600] = H
        elif kind == "first_tile":
            buf[s0 + 700] = L
    fixed = oracle.to_well_formed_batch(buf, off)
    t_off = offsets_dev(off)
    b = off.size - 1
    res = torch.empty(b, dtype=torch.uint8, device="cuda")
    want1 = oracle.is_well_formed_batch(buf, off)
    assert int((want1 == 0).sum()) > 50
    want2 = oracle.is_well_formed_batch(fixed, off)
    assert want2.all()
    t1, _ = to_dev(buf, 0, pad=8)
    t2, _ = to_dev(fixed, 0, pad=8)
    for rows in ROWS:
        # many waves with a tile or two each, and few waves with long runs
        # of tiles (where a wave reads a clean tile of a string before the
        # erring one and publishes the clearing device-wide)
        for wg_waves, grid in ((4, 8), (1, 64), (1, 1)):
            wf.set_params(wf.OP_IS, 1, -1, rows=rows, wg_waves=wg_waves, grid_per_cu=grid, nontemporal=0)
            for hint in (0, int(off[-1])):
                for t, want, what in ((t1, want1, "ill-formed"), (t2, want2, "repaired"), (t1, want1, "again")):
                    wf.utf16wf_batch(wf.OP_IS, t, t_off, results=res, units_hint=hint)
                    got = res.cpu().numpy()
                    assert np.array_equal(got, want), \
                        f"rows={rows} waves={wg_waves} grid={grid} hint={hint} {what}: {np.nonzero(got != want)[0][:10]}"
    wf.reset_params()


def test_locate_few_long_strings_workgroup_totals(wf):
    """Locate over batches of few long strings with errors throughout: waves
    that end on the same string add their totals in their workgroup first.
    Shapes with more waves than tiles leave idle waves in a workgroup, which
    must still report; a shape with one wave per workgroup has nothing to
    combine."""
    torch = torch_mod()
    rng = np.random.default_rng(21)
    cases = []
    for lens in ([1_000_000], [700_000, 3, 900_001], [0, 250_000, 0, 250_000, 1], [5] * 40 + [600_000]):
        lens = np.array(lens, np.int64)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        buf = W.mix(int(off[-1]), 1e-2, int(rng.integers(1 << 30)))
        cases.append((buf, off))
    for rows, wg_waves, grid in ((4, 16, 64), (8, 4, 8), (1, 1, 32), (2, 16, 1)):
        for batch in (0, 1):  # a locate over few strings takes the flat parameters
            wf.set_params(wf.OP_LOCATE, batch, -1, rows=rows, wg_waves=wg_waves, grid_per_cu=grid, nontemporal=0)
        for buf, off in cases:
            t_in, _ = to_dev(buf, 0, pad=8)
            t_off = offsets_dev(off)
            b = off.size - 1
            first = torch.empty(b, dtype=torch.int64, device="cuda")
            cnt = torch.empty(b, dtype=torch.int64, device="cuda")
            want_first, want_cnt = oracle.locate_batch(buf, off)
            for hint in (0, int(off[-1])):
                wf.utf16wf_batch(wf.OP_LOCATE, t_in, t_off, first=first, count=cnt, units_hint=hint)
                what = f"rows={rows} waves={wg_waves} grid={grid} lens={np.diff(off)[:3]}.. hint={hint}"
                assert np.array_equal(first.cpu().numpy(), want_first), f"first {what}"
                assert np.array_equal(cnt.cpu().numpy(), want_cnt), f"count {what}"
    wf.reset_params()


def test_runs_of_empty_strings(wf):
    """Runs of empty strings (equal offsets) of every length around the
    64-offset scan step and far beyond it: at the batch's start, inside a
    tile, at a tile edge, at the end, and between two runs; a run's position
    belongs to the non-empty string after it."""
    torch = torch_mod()
    rng = np.random.default_rng(31)
    n = 40_000
    buf = W.mix(n, 2e-2, 17)
    for rows in (1, 4):
        T = 512 * rows
        for run in (1, 63, 64, 65, 127, 128, 129, 1000, 200_000):
            cuts = [0, 0, 700, T, 2 * T + 5, n // 2, n - 1, n, n]
            offs = [0]
            for c in cuts[1:]:
                offs.extend([c] * (run if c in (0, T, n // 2, n) else 1))
            offs.append(n)
            off = np.array(sorted(offs), np.int64)
            _force_rows(wf, rows)
            _check_batch(wf, buf, off, what=f"runs of {run} empty, rows={rows}")
            _check_batch(wf, buf, off, what=f"runs of {run} empty, rows={rows}, hinted", hint=n)
    wf.reset_params()
    # a run of a million empty strings before one long string (its time is
    # reported by the benchmark, not asserted here)
    big = W.mix(1 << 22, 1e-3, 18)
    off = np.concatenate([np.zeros(1_000_000, np.int64), [0, big.size]]).astype(np.int64)
    _check_batch(wf, big, off, what="1M empty strings first", hint=big.size)


def test_random_shapes_and_contents(wf):
    """Random launch shapes (rows, waves per workgroup, workgroups per CU,
    non-temporal, in-place store mode) against random batches: long and short strings, runs of
    empty strings, error-free strings, strings with one late error and with
    dense errors; every operation, with and without a size hint, against
    the oracle."""
    rng = np.random.default_rng(2026)
    alphabet = np.array([A, 0x4E2D, H, L], np.uint16)
    for case in range(24):
        parts, lens = [], []
        for _ in range(int(rng.integers(1, 40))):
            kind = int(rng.integers(0, 6))
            if kind == 0:    # a run of empty strings
                lens.extend([0] * int(rng.choice([1, 63, 64, 65, 300])))
                continue
            n = int(rng.choice([1, 7, 100, 2048, 5000, 30_000, 120_000]))
            s = np.full(n, A, np.uint16)
            if kind == 1:    # random units, errors everywhere
                s = alphabet[rng.integers(0, alphabet.size, size=n)].astype(np.uint16)
            elif kind == 2:  # one error late
                s[int(n * 0.9)] = H if rng.random() < 0.5 else L
            elif kind == 3:  # dense errors past the first 600 units
                s[600::97] = L
            parts.append(s)
            lens.append(n)
        buf = np.concatenate(parts) if parts else np.full(1, A, np.uint16)
        lens = np.array(lens, np.int64)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        if off[-1] > buf.size:
            buf = np.concatenate([buf, np.full(int(off[-1]) - buf.size, A, np.uint16)])
        rows = int(rng.choice([1, 2, 4, 8]))
        wg_waves = int(rng.choice([1, 2, 4, 8, 16]))
        grid = int(rng.choice([1, 2, 8, 32, 64]))
        nt = int(rng.integers(0, 2))
        sl = (case // 2) % 2  # in-place store mode: whole lines or changed vectors
        _force_rows(wf, rows, wg_waves, grid, nt, store_lines=sl)
        hint = int(off[-1]) if case % 2 else 0
        _check_batch(wf, buf, off, what=f"case {case} rows={rows} waves={wg_waves} grid={grid} nt={nt} lines={sl}",
                     hint=hint)
    wf.reset_params()
