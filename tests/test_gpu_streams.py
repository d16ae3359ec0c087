"""Calls captured into a graph by the caller, and calls racing on several
streams: results stay exact."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2601_06349_amd import workloads as W
from tests.gpu_util import assert_same, offsets_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wf():
    torch_mod()
    import paper_2601_06349_amd as wf
    wf.reset_params()
    return wf


def test_caller_graph_capture_and_replay(wf):
    """The flat calls initialise their results with kernels (no memset nodes),
    so a caller can capture them; every replay, with new input contents and
    eager work in between, equals the oracle."""
    torch = torch_mod()
    rng = np.random.default_rng(3)
    n = 300_001
    base = W.mix(n, 1e-3, 31)
    x = torch.from_numpy(base.view(np.int16)).cuda()
    y = torch.empty_like(x)
    res = torch.empty(1, dtype=torch.int32, device="cuda")
    loc = torch.empty(2, dtype=torch.int64, device="cuda")
    # warm up outside the capture (first calls query the device)
    wf.utf16_to_well_formed(x, y)
    wf.utf16_is_well_formed(x, res)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        wf.utf16_to_well_formed(x, y)
        wf.utf16_is_well_formed(x, res)
        wf.lib().utf16_locate_ill_formed(x.data_ptr(), n, loc.data_ptr(), loc.data_ptr() + 8,
                                         torch.cuda.current_stream().cuda_stream)
    for rep in range(5):
        cur = base.copy()
        if rep % 2:
            cur = oracle.to_well_formed(cur)  # a well-formed input on odd replays
        cur[rng.integers(0, n, size=rep * 7)] = 0xDC00
        x.copy_(torch.from_numpy(cur.view(np.int16)))
        y.fill_(0)
        res.fill_(7)
        loc.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        want, cnt = oracle.to_well_formed_count(cur)
        assert_same(to_host(y), want, f"replay {rep}")
        assert int(res.item()) == int(cnt == 0), f"is replay {rep}"
        l = loc.cpu().numpy()
        assert int(l[1]) == cnt and int(l[0]) == oracle.first_bad(cur), f"locate replay {rep}"


def test_concurrent_streams(wf):
    torch = torch_mod()
    streams = [torch.cuda.Stream() for _ in range(4)]
    inputs = [W.mix(1_000_003 + 17 * i, 1e-2, 50 + i) for i in range(4)]
    d_in = [torch.from_numpy(s.view(np.int16)).cuda() for s in inputs]
    d_out = [torch.empty_like(x) for x in d_in]
    batches = [W.ragged_batch(b=20_000, seed=60 + i) for i in range(4)]
    d_b = [(torch.from_numpy(b.view(np.int16)).cuda(), offsets_dev(o)) for b, o in batches]
    d_bo = [torch.empty_like(b) for b, _ in d_b]
    res = [torch.empty(o.numel() - 1, dtype=torch.uint8, device="cuda") for _, o in d_b]
    torch.cuda.synchronize()
    for _ in range(10):
        for i, st in enumerate(streams):
            with torch.cuda.stream(st):
                wf.utf16_to_well_formed(d_in[i], d_out[i])
                wf.utf16_to_well_formed_batch(d_b[i][0], d_b[i][1], out=d_bo[i])
                wf.utf16_is_well_formed_batch(d_b[i][0], d_b[i][1], results=res[i])
    torch.cuda.synchronize()
    for i in range(4):
        assert_same(to_host(d_out[i]), oracle.to_well_formed(inputs[i]), f"stream {i} flat")
        b, o = batches[i]
        assert_same(to_host(d_bo[i]), oracle.to_well_formed_batch(b, o), f"stream {i} batch")
        assert np.array_equal(res[i].cpu().numpy(), oracle.is_well_formed_batch(b, o))
