"""utf16wf_validate_batch_noalloc (the batch validation that allocates
nothing, its flag in static device memory) against utf16wf_validate_batch,
through the C ABI: the same status for valid batches, bad offsets and
overlapping buffers, on calls in a row whose inputs shrink, so a flag left
set by one call must not leak into the next."""
from __future__ import annotations

import numpy as np
import pytest

from tests.gpu_util import log, offsets_dev, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = torch_mod()
    import paper_2601_06349_amd as wf
    return torch, wf, wf.lib()


def _both(L, stream, *args):
    """(existing entry point's status, no-alloc entry point's status)."""
    a = L.utf16wf_validate_batch(*args, stream)
    b = L.utf16wf_validate_batch_noalloc(*args, stream)
    return a, b


def _cases(torch, b, seed):
    """Valid and invalid batches of b strings over one buffer."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 200, size=b)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n = int(off[-1])
    buf = torch.zeros(n + 64, dtype=torch.int16, device="cuda")
    far = torch.zeros(n + 64, dtype=torch.int16, device="cuda")
    dec = off.copy()
    dec[b // 2] = dec[b // 2 + 1] + 1  # one offset above its successor
    past = off.copy()
    past[-1] = buf.numel() + 1  # beyond the buffer
    neg = off.copy()
    neg[0] = -1
    return buf, far, n, {"valid": off, "decreasing": dec, "past the end": past, "negative": neg}


def test_noalloc_validation_matches(env):
    torch, wf, L = env
    stream = torch.cuda.current_stream().cuda_stream
    want_codes = {"valid": wf.OK, "decreasing": wf.EOFFSETS, "past the end": wf.EOFFSETS, "negative": wf.EOFFSETS}
    calls = 0
    for b, seed in ((1_000_000, 1), (1000, 2), (1, 3)):  # each round smaller than the one before
        buf, far, n, cases = _cases(torch, b, seed)
        P = buf.data_ptr()
        for name, off in cases.items():
            t_off = offsets_dev(off)
            for out, label in ((far.data_ptr(), "distinct"), (P, "in place"), (None, "no output")):
                log(f"validate b={b} {name} {label}")
                a, c = _both(L, stream, P, out, t_off.data_ptr(), b, buf.numel())
                assert a == c == want_codes[name], (b, name, label, a, c)
                calls += 1
            if name == "valid" and n >= 4:
                # out two units past in: the spans overlap
                a, c = _both(L, stream, P, P + 4, t_off.data_ptr(), b, buf.numel())
                assert a == c == wf.EOVERLAP, (b, "overlap", a, c)
                # out just past the span: no overlap
                a, c = _both(L, stream, P, P + 2 * n, t_off.data_ptr(), b, buf.numel() + n)
                assert a == c == wf.OK, (b, "adjacent", a, c)
        # a bad call followed by a good one of the same size: the flag is cleared
        bad = offsets_dev(cases["decreasing"])
        good = offsets_dev(cases["valid"])
        assert L.utf16wf_validate_batch_noalloc(P, None, bad.data_ptr(), b, buf.numel(), stream) == wf.EOFFSETS
        assert L.utf16wf_validate_batch_noalloc(P, None, good.data_ptr(), b, buf.numel(), stream) == wf.OK
    # argument errors are the existing entry point's
    for args in ((None, None, 0x1000, 3, 10), (0x1001, None, 0x1000, 3, 10), (0x1000, None, 0x1004, 3, 10),
                 (0x1000, None, 0x1000, -1, 10)):
        assert L.utf16wf_validate_batch(*args, None) == L.utf16wf_validate_batch_noalloc(*args, None) < 0
    log(f"{calls} comparisons")
