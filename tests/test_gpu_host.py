"""Host-resident input: the chunked, overlapped copy-in / repair / copy-out
path equals the oracle, for chunk edges that split pairs, in place and with
pinned host memory."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2601_06349_amd import workloads as W
from tests.gpu_util import assert_same, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wf():
    torch_mod()
    import paper_2601_06349_amd as wf
    return wf


@pytest.mark.parametrize("chunk", [1, 2, 7, 1000, 4097, 0])
def test_host_chunks(wf, chunk):
    rng = np.random.default_rng(chunk)
    alphabet = np.array([0x41, 0xD801, 0xDC02, 0xDBFF, 0xDFFF], np.uint16)
    for n in (1, 2, 3, 999, 1000, 1001, 20_011):
        if chunk in (1, 2) and n > 1001:
            continue
        s = alphabet[rng.integers(0, alphabet.size, size=n)]
        want = oracle.to_well_formed(s)
        assert_same(wf.utf16_to_well_formed_host(s, chunk_units=chunk), want, f"host n={n} chunk={chunk}")
        t = s.copy()
        wf.utf16_to_well_formed_host(t, out=t, chunk_units=chunk)
        assert_same(t, want, f"host in place n={n} chunk={chunk}")


def test_host_pinned_large(wf):
    torch = torch_mod()
    s = W.mix(50_000_017, 1e-3, 77)
    want = oracle.to_well_formed(s)
    pin_in = torch.empty(s.size, dtype=torch.int16, pin_memory=True)
    pin_out = torch.empty(s.size, dtype=torch.int16, pin_memory=True)
    a = pin_in.numpy().view(np.uint16)
    b = pin_out.numpy().view(np.uint16)
    a[:] = s
    wf.utf16_to_well_formed_host(a, out=b, chunk_units=1 << 22)
    assert_same(b, want, "pinned")
    wf.utf16_to_well_formed_host(a, out=a)
    assert_same(a, want, "pinned in place")

