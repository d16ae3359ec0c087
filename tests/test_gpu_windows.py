"""The GPU's unit classification, exhaustively: every window of three units
whose top six bits take all 64^3 combinations (random low ten bits), each
window followed by an ASCII unit, through the flat kernels at every input
phase and through the batch kernels (each window a string of its own, and
all windows as one string), against the oracle. A unit's result depends only
on its two neighbours (Sec. 3.1, the block formulation), so this covers
every case of the per-unit rule the kernels implement."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.gpu_util import assert_same, log, offsets_dev, to_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu

SENTINEL = 0x1234


def window_string(seed=11):
    """All 64^3 three-unit windows of top-6-bit classes with random low bits,
    each followed by 'A' (the same string the oracle's exhaustive pin uses)."""
    rng = np.random.default_rng(seed)
    cls = np.arange(64, dtype=np.uint32)
    a, b, c = np.meshgrid(cls, cls, cls, indexing="ij")
    win = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)
    units = (win << 10) | rng.integers(0, 1024, size=win.shape).astype(np.uint32)
    s = np.full((win.shape[0], 4), 0x0041, dtype=np.uint32)
    s[:, :3] = units
    return s.ravel().astype(np.uint16)


@pytest.fixture(scope="module")
def wf():
    torch_mod()
    import paper_2601_06349_amd as wf
    wf.reset_params()
    yield wf
    wf.reset_params()


@pytest.fixture(scope="module")
def windows():
    s = window_string()
    assert s.size == 4 * 64 ** 3
    return s


def _shapes(wf):
    """The built-in shapes and the tuned ones (when a cache exists)."""
    from paper_2601_06349_amd import tune
    wf.reset_params()
    yield "defaults"
    if tune.apply_cache() is not None:
        yield "tuned"
    wf.reset_params()


def test_windows_flat_every_phase(wf, windows):
    want, cnt = oracle.to_well_formed_count(windows)
    for shape in _shapes(wf):
        for phase in range(8):
            log(f"windows flat, {shape}, phase {phase}")
            t_in, _ = to_dev(windows, phase, pad=8)
            t_out, _ = to_dev(np.full(windows.size, SENTINEL, np.uint16), (phase + 5) % 8 if phase % 2 else phase,
                              pad=8)
            wf.utf16_to_well_formed(t_in, t_out)
            assert_same(to_host(t_out), want, f"windows flat {shape} phase {phase}")
            wf.utf16_to_well_formed_inplace(t_in)
            assert_same(to_host(t_in), want, f"windows in place {shape} phase {phase}")
            t_in, _ = to_dev(windows, phase, pad=8)
            loc = wf.utf16_locate_ill_formed(t_in).cpu().numpy()
            assert int(loc[0]) == oracle.first_bad(windows) and int(loc[1]) == cnt


def _batch_vs_oracle(wf, buf, off, what):
    torch = torch_mod()
    b = off.size - 1
    t_in = torch.from_numpy(buf.view(np.int16)).cuda()
    t_off = offsets_dev(off)
    t_out = torch.full_like(t_in, SENTINEL)
    for hint in (0, buf.size):
        log(f"{what}, hint {hint}")
        t_out.fill_(SENTINEL)
        wf.utf16wf_batch(wf.OP_TO, t_in, t_off, out=t_out, units_hint=hint)
        assert_same(to_host(t_out), oracle.to_well_formed_batch(buf, off), f"{what} repair, hint {hint}")
        res = torch.empty(b, dtype=torch.uint8, device="cuda")
        wf.utf16wf_batch(wf.OP_IS, t_in, t_off, results=res, units_hint=hint)
        assert np.array_equal(res.cpu().numpy(), oracle.is_well_formed_batch(buf, off)), f"{what} check"
        first = torch.empty(b, dtype=torch.int64, device="cuda")
        count = torch.empty(b, dtype=torch.int64, device="cuda")
        wf.utf16wf_batch(wf.OP_LOCATE, t_in, t_off, first=first, count=count, units_hint=hint)
        want_f, want_c = oracle.locate_batch(buf, off)
        assert np.array_equal(first.cpu().numpy(), want_f) and np.array_equal(count.cpu().numpy(), want_c), what


def test_windows_batch(wf, windows):
    n = windows.size
    cases = {
        # each window with its ASCII unit a string of its own
        "4-unit strings": np.arange(0, n + 1, 4, dtype=np.int64),
        # each window alone (3 units), the ASCII units strings of one unit
        "3-unit windows": np.sort(np.concatenate([np.arange(0, n + 1, 4), np.arange(3, n, 4)])).astype(np.int64),
        "one string": np.array([0, n], dtype=np.int64),
    }
    for shape in _shapes(wf):
        for name, off in cases.items():
            _batch_vs_oracle(wf, windows, off, f"windows batch {name}, {shape}")
