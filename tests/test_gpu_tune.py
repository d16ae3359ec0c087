"""The autotuner on the GPU, over one flat size class with the quick grid:
it writes a cache of valid launch shapes (the in-place repair's with a store
mode), none slower than the default in the tuner's own timing, and that
cache loads back into the library."""
from __future__ import annotations

import json

import pytest

from tests.gpu_util import log, torch_mod

pytestmark = pytest.mark.gpu


def test_quick_tune_one_flat_class(tmp_path):
    torch_mod()
    import paper_2601_06349_amd as wf
    from paper_2601_06349_amd import tune

    out = tmp_path / "cache.json"
    try:
        data = tune.tune(quick=True, flat_classes=[16], out=str(out), log=log, batches=False)
        entries = data["entries"]
        assert sorted(e["op"] for e in entries) == sorted([wf.OP_IS, wf.OP_TO, wf.OP_TO_INPLACE, wf.OP_LOCATE])
        for e in entries:
            p = e["params"]
            assert e["batch"] == 0 and e["size_class"] == 16
            assert p["rows"] in (1, 2, 4, 8) and 1 <= p["wg_waves"] <= 16 and 1 <= p["grid_per_cu"] <= 64
            assert p["nontemporal"] in (0, 1) and p["store_lines"] in (0, 1)
            assert e["tuned_ms"] <= e["default_ms"] * 1.0001
        assert json.loads(out.read_text())["entries"] == entries
        wf.reset_params()
        assert tune.apply_cache(str(out)) == "cache.json"
        for e in entries:
            assert wf.get_params(e["op"], 0, 1 << 16) == e["params"]
            # a class without an entry takes the nearest tuned one
            assert wf.get_params(e["op"], 0, 1 << 20) == e["params"]
    finally:
        wf.reset_params()
