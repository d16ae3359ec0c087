"""Helpers shared by the GPU parity tests (no test functions here)."""
from __future__ import annotations

import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_mod():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test started without a visible GPU")
    return torch


def to_dev(arr: np.ndarray, phase: int = 0, pad: int = 0):
    """Device int16 tensor holding ``arr`` whose data pointer sits ``phase``
    units past a 16-byte boundary (a view into a larger allocation), with
    ``pad`` sentinel units (0x1234) on both sides in the allocation."""
    torch = torch_mod()
    arr = np.ascontiguousarray(arr, dtype=np.uint16)
    n = arr.size
    pad = (pad + 7) // 8 * 8
    base = torch.full((n + phase + 2 * pad + 16,), 0x1234, dtype=torch.int16, device="cuda")
    start = phase + pad
    # torch allocations are 256-byte aligned, so `start` units in gives phase
    view = base[start:start + n]
    if n:
        assert (view.data_ptr() - base.data_ptr()) == 2 * start
        assert (base.data_ptr() & 15) == 0
        assert (view.data_ptr() & 15) == (2 * phase) % 16
        view.copy_(torch.from_numpy(arr.view(np.int16)))
    return view, base


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint16)


def offsets_dev(off: np.ndarray):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).to("cuda")


def assert_same(got: np.ndarray, want: np.ndarray, what=""):
    if got.shape != want.shape:
        raise AssertionError(f"{what}: shape {got.shape} != {want.shape}")
    diff = np.nonzero(got != want)[0]
    if diff.size:
        i = int(diff[0])
        lo, hi = max(0, i - 3), min(got.size, i + 4)
        raise AssertionError(
            f"{what}: {diff.size} units differ, first at {i}: got {[hex(x) for x in got[lo:hi]]} "
            f"want {[hex(x) for x in want[lo:hi]]}")
