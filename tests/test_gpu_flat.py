"""GPU parity of the flat (single-buffer) entry points against the CPU oracle.

Everything is integer work, so the bar is bit-exact equality. All calls go
through the C ABI (via the ctypes binding)."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from paper_2601_06349_amd import workloads as W
from tests import oracle_pins as P
from tests.gpu_util import assert_same, log, to_dev, to_host, torch_mod

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
        wf.set_params(op, 0, -1, rows=rows, wg_waves=wg_waves, grid_per_cu=grid_per_cu, nontemporal=nt,
                      store_lines=store_lines)


def _check_all(wf, s, phase_in=0, phase_out=0, what=""):
    """OOP, in place, is and locate on s vs the oracle."""
    torch = torch_mod()
    want, cnt = oracle.to_well_formed_count(s)
    t_in, _ = to_dev(s, phase_in, pad=8)
    t_out, base_out = to_dev(np.zeros(s.size, np.uint16), phase_out, pad=8)
    before = to_host(base_out)
    wf.utf16_to_well_formed(t_in, t_out)
    got = to_host(t_out)
    assert_same(got, want, f"oop {what} phase {phase_in}/{phase_out}")
    # nothing outside the output range was written
    after = to_host(base_out)
    start = phase_out + 8
    assert np.array_equal(after[:start], before[:start]) and np.array_equal(after[start + s.size:],
                                                                            before[start + s.size:])
    # in place
    t_ip, base_ip = to_dev(s, phase_in, pad=8)
    before_ip = to_host(base_ip)
    wf.utf16_to_well_formed_inplace(t_ip)
    assert_same(to_host(t_ip), want, f"inplace {what} phase {phase_in}")
    after_ip = to_host(base_ip)
    st = phase_in + 8
    assert np.array_equal(after_ip[:st], before_ip[:st]) and np.array_equal(after_ip[st + s.size:],
                                                                            before_ip[st + s.size:])
    # is / locate
    assert wf.is_well_formed(t_in) == oracle.is_well_formed(s), f"is {what}"
    loc = wf.utf16_locate_ill_formed(t_in).cpu().numpy()
    assert int(loc[0]) == oracle.first_bad(s), f"first_bad {what}"
    assert int(loc[1]) == cnt, f"count {what}"
    torch.cuda.synchronize()


def test_fig3_example(wf):
    inp, out = P.load_fig3()
    for phase in range(8):
        t, _ = to_dev(inp, phase, pad=8)
        assert_same(to_host(wf.utf16_to_well_formed(t)), out, f"fig3 phase {phase}")
        assert not wf.is_well_formed(t)
    # the example planted at many offsets of a larger all-ASCII context
    for off in (0, 1, 7, 8, 9, 500, 511, 512, 1020, 2040, 2047, 4090, 4096):
        s = np.full(8192 + 64, A, np.uint16)
        s[off:off + inp.size] = inp
        _check_all(wf, s, what=f"fig3@{off}")


def test_readme_example(wf):
    """The usage example in the README gives the values it states."""
    torch = torch_mod()
    s = torch.tensor([0x48, 0xD800, 0x69, 0xDC00], dtype=torch.uint16, device="cuda")
    assert wf.utf16_to_well_formed(s).cpu().tolist() == [0x48, 0xFFFD, 0x69, 0xFFFD]
    assert wf.is_well_formed(s) is False
    buf = torch.tensor([0xD83D, 0xDE0A, 0xD83D, 0xDE0A], dtype=torch.uint16, device="cuda")
    off = torch.tensor([0, 1, 4], dtype=torch.int64, device="cuda")
    assert wf.utf16_to_well_formed_batch(buf, off).cpu().tolist() == [0xFFFD, 0xFFFD, 0xD83D, 0xDE0A]
    res = torch.empty(2, dtype=torch.uint8, device="cuda")
    wf.utf16wf_batch(wf.OP_IS, buf, off, results=res, units_hint=4)
    assert res.cpu().tolist() == [0, 0]


def test_small_workload(wf):
    s = W.small_string()
    log(f"small workload n={s.size}")
    for rows in ROWS:
        _force_rows(wf, rows)
        _check_all(wf, s, what=f"small rows={rows}")
    wf.reset_params()
    _check_all(wf, s, what="small default")


SIZES = [0, 1, 2, 3, 7, 8, 9, 15, 16, 17, 63, 64, 65, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 4095,
         4096, 4097, 8191, 8193, 65537, 100003]


@pytest.mark.parametrize("rows", ROWS)
def test_sizes_and_phases(wf, rows):
    _force_rows(wf, rows)
    rng = np.random.default_rng(100 + rows)
    alphabet = np.array([A, 0x4E2D, H, L, 0xDBFF, 0xDFFF, 0xFFFD], np.uint16)
    for n in SIZES:
        s = alphabet[rng.integers(0, alphabet.size, size=n)] if n else np.zeros(0, np.uint16)
        phases = [(0, 0), (1, 1), (3, 5), (7, 0)] if n < 5000 else [(0, 0), (5, 2)]
        for pi, po in phases:
            _check_all(wf, s, pi, po, what=f"n={n} rows={rows}")
    wf.reset_params()


@pytest.mark.parametrize("rows", ROWS)
def test_every_output_phase(wf, rows):
    """Output at every address phase against two input phases (all seven
    relative shifts of the realigned stores, and equal phases), over several
    tiles with partial ends, dense surrogates; nothing outside the output
    range is written."""
    _force_rows(wf, rows)
    rng = np.random.default_rng(300 + rows)
    alphabet = np.array([A, H, L, 0xDBFF, 0xDC00, 0x4E2D], np.uint16)
    for n in (1, 7, 9, 3 * 512 * rows + 37, 5 * 512 * rows - 3):
        s = alphabet[rng.integers(0, alphabet.size, size=n)]
        for pi in (0, 3):
            for po in range(8):
                _check_all(wf, s, pi, po, what=f"n={n} rows={rows}")
    wf.reset_params()


PATTERNS = [[H], [L], [H, L], [L, H], [H, H, L], [H, L, L], [L, L], [H, H]]


@pytest.mark.parametrize("rows", ROWS)
def test_patterns_at_every_lane_boundary(wf, rows):
    """Each pattern planted across every 8-unit lane boundary (so across every
    row, tile, wave and workgroup boundary too), at four offsets."""
    _force_rows(wf, rows)
    n = 3 * 4096 + 37
    for pat, d in itertools.product(PATTERNS, (-2, -1, 0, 1)):
        s = np.full(n, A, np.uint16)
        for b in range(0, n, 8):
            p = b + d
            if 0 <= p and p + len(pat) <= n:
                s[p:p + len(pat)] = pat
        _check_all(wf, s, what=f"pattern {pat} d={d} rows={rows}")
    wf.reset_params()


def test_single_plants_decide_is(wf):
    n = 3 * 4096 + 5
    for rows in ROWS:
        _force_rows(wf, rows)
        for p in (0, 1, 7, 8, 511, 512, 1023, 1024, 2047, 2048, 4095, 4096, n - 2):
            for pat, ok in (([H, L], True), ([H], False), ([L], False), ([L, H], False)):
                if p + len(pat) > n:
                    continue
                s = np.full(n, A, np.uint16)
                s[p:p + len(pat)] = pat
                t, _ = to_dev(s)
                assert wf.is_well_formed(t) == ok, (rows, p, pat)
                loc = wf.utf16_locate_ill_formed(t).cpu().numpy()
                assert int(loc[0]) == oracle.first_bad(s)
        s = np.full(n, A, np.uint16)
        s[-1] = H
        t, _ = to_dev(s)
        assert not wf.is_well_formed(t)
    wf.reset_params()


@pytest.mark.parametrize("combo", list(itertools.product((1, 4, 16), (1, 8), (0, 1))))
def test_launch_shapes(wf, combo):
    wg, gpc, nt = combo
    s = W.mix(200_003, 1e-2, 77)
    s[1000:1100] = W.all_surrogates(100, 5)
    for rows in ROWS:
        _force_rows(wf, rows, wg_waves=wg, grid_per_cu=gpc, nt=nt)
        _check_all(wf, s, 0, 0, what=f"shape rows={rows} wg={wg} gpc={gpc} nt={nt}")
    wf.reset_params()


@pytest.mark.parametrize("store_lines", [1, 0])
def test_inplace_store_modes(wf, store_lines):
    """In-place repair in both store modes (whole 128-byte lines holding a
    change, or only the 16-byte vectors that changed), every row count, at
    several phases: equal to the oracle, nothing outside the string
    written."""
    s = W.mix(300_007, 1e-2, 81)
    s[5000:7000] = W.all_surrogates(2000, 6)
    want = oracle.to_well_formed(s)
    for rows in ROWS:
        _force_rows(wf, rows, store_lines=store_lines)
        for ph in (0, 3, 7):
            t, base = to_dev(s, ph, pad=8)
            before = to_host(base)
            wf.utf16_to_well_formed_inplace(t)
            got = to_host(base)
            lo = ph + 8
            assert_same(got[lo:lo + s.size], want, f"in place rows={rows} lines={store_lines} phase={ph}")
            assert np.array_equal(got[:lo], before[:lo]) and np.array_equal(got[lo + s.size:], before[lo + s.size:])
    wf.reset_params()


def test_copy_kernel(wf):
    torch = torch_mod()
    s = W.mix(1_000_001, 1e-3, 3)
    for ph in (0, 3):
        t, _ = to_dev(s, ph, pad=8)
        o, _ = to_dev(np.zeros_like(s), ph, pad=8)
        wf.utf16wf_copy_units(t, o)
        torch.cuda.synchronize()
        assert_same(to_host(o), s, "copy")


@pytest.mark.parametrize("variant", W.SINGLE_VARIANTS)
def test_single_buffer_full_size(wf, variant):
    """The 268,435,456-unit buffers at full size, default launch shape (the
    one the benchmark times): out of place, in place, is, locate."""
    torch = torch_mod()
    from paper_2601_06349_amd import tune
    tune.apply_cache()  # the launch shapes the benchmark uses
    log(f"generating {variant}")
    s = W.single_buffer(variant)
    want, cnt = oracle.to_well_formed_count(s)
    log(f"{variant}: oracle replaced {cnt}")
    t_in = torch.from_numpy(s.view(np.int16)).to("cuda")
    t_out = torch.empty_like(t_in)
    wf.utf16_to_well_formed(t_in, t_out)
    assert_same(to_host(t_out), want, f"{variant} oop")
    assert wf.is_well_formed(t_in) == (cnt == 0)
    loc = wf.utf16_locate_ill_formed(t_in).cpu().numpy()
    assert int(loc[1]) == cnt and int(loc[0]) == oracle.first_bad(s)
    wf.utf16_to_well_formed_inplace(t_in)
    assert_same(to_host(t_in), want, f"{variant} inplace")
    assert wf.is_well_formed(t_in)
    if variant == "allsur":
        assert abs(cnt / s.size - 0.5) < 0.01  # about half of the units pair up
    del t_in, t_out
    torch.cuda.empty_cache()
    wf.reset_params()


def test_beyond_32bit_indices(wf):
    """A buffer of 2^31 + 2^20 + 3 units (4.3 GB): mismatches planted around
    unit 2^31 and near the end; outputs checked on windows against the oracle
    (a unit's result depends only on its two neighbours, so a window with one
    unit of margin on each side is exact)."""
    torch = torch_mod()
    n = (1 << 31) + (1 << 20) + 3
    t = torch.full((n,), A, dtype=torch.int16, device="cuda")
    plants = {(1 << 31) - 2: [H, H, L], (1 << 31) + 7: [L], (1 << 31) + 4096: [H, L], n - 3: [L, H, H],
              (1 << 30) + 1: [H]}
    for p, pat in plants.items():
        t[p:p + len(pat)] = torch.tensor(np.array(pat, np.uint16).view(np.int16), device="cuda")
    out = torch.empty_like(t)
    wf.utf16_to_well_formed(t, out)
    assert not wf.is_well_formed(t)
    loc = wf.utf16_locate_ill_formed(t).cpu().numpy()
    host_windows = {}
    for p in plants:
        a, b = max(0, p - 64), min(n, p + 64)
        host_windows[p] = (a, b, to_host(t[a:b]))
    bad_units = set()
    for p, (a, b, s) in sorted(host_windows.items()):
        ctx_a, ctx_b = a - (1 if a > 0 else 0), b + (1 if b < n else 0)
        s_ctx = to_host(t[ctx_a:ctx_b])
        w = oracle.to_well_formed(s_ctx)[a - ctx_a:a - ctx_a + (b - a)]
        assert_same(to_host(out[a:b]), w, f"window at {p}")
        bad_units.update(a + int(i) for i in np.nonzero(w != s)[0])
    assert len(bad_units) == 6
    assert int(loc[1]) == len(bad_units) and int(loc[0]) == min(bad_units)
    wf.utf16_to_well_formed_inplace(t)
    for p, (a, b, s) in host_windows.items():
        assert_same(to_host(t[a:b]), to_host(out[a:b]), f"in place window at {p}")
    assert wf.is_well_formed(t)
    # a batch whose offsets pass 2^31
    t2 = out  # reuse: fill with a known pattern
    t2.fill_(A)
    t2[(1 << 31) - 2] = H - 65536
    t2[(1 << 31) - 1] = L - 65536
    cut = np.array([0, (1 << 31) - 1, (1 << 31) + 5, n], np.int64)
    offs = torch.from_numpy(cut).cuda()
    res = wf.utf16_is_well_formed_batch(t2, offs).cpu().numpy()
    assert list(res) == [0, 0, 1]  # the pair is cut by the offset at 2^31 - 1
    wf.utf16_to_well_formed_batch_inplace(t2, offs)
    assert list(to_host(t2[(1 << 31) - 3:(1 << 31) + 1])) == [A, 0xFFFD, 0xFFFD, A]
    del t, out, t2
    torch.cuda.empty_cache()
