"""C-ABI tests that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before making any HIP call."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(utf16\w*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2601_06349_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libutf16wf.so is not built (run python -m paper_2601_06349_amd.build)")
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert len(names) >= 20, names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"
    from paper_2601_06349_amd import _lib
    assert set(names) <= set(_lib.SIGNATURES), "binding is missing a declared function"


def test_headers_compile_as_c(tmp_path):
    """The headers are a C ABI: they compile as C99 with warnings as errors,
    and calls through them type-check."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(
        '#include "utf16wf.h"\n#include "utf16wf_serve.h"\n'
        "int use(const uint16_t *in, uint16_t *out, int64_t n, const int64_t *off, uint8_t *res, void *s) {\n"
        "    utf16wf_params p;\n"
        "    int rc = utf16_to_well_formed(in, out, n, s);\n"
        "    rc |= utf16_is_well_formed_batch(in, off, 3, res, s);\n"
        "    rc |= utf16wf_get_params(UTF16WF_OP_TO, 0, n, &p);\n"
        "    utf16wf_serve_config c = {4, UTF16WF_OP_TO, 1 << 30, 64, 1 << 20, 0, 0};\n"
        "    (void)c;\n"
        "    return rc | utf16wf_abi_version();\n"
        "}\n")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", HEADER_DIR, "-c",
                        str(src), "-o", str(tmp_path / "use.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_abi_version(L):
    assert L.utf16wf_abi_version() == 2


def _rc(L, name, *args):
    return getattr(L, name)(*args)


A = 0x10000  # a fake, never dereferenced, 16-byte aligned address


def test_flat_argument_errors(L):
    from paper_2601_06349_amd import EALIGN, EINVAL, EOVERLAP
    assert _rc(L, "utf16_to_well_formed", A, A + 4096, -1, None) == EINVAL
    assert _rc(L, "utf16_to_well_formed", None, A, 5, None) == EINVAL
    assert _rc(L, "utf16_to_well_formed", A, None, 5, None) == EINVAL
    assert _rc(L, "utf16_to_well_formed", A + 1, A + 4096, 5, None) == EALIGN
    assert _rc(L, "utf16_to_well_formed", A, A + 4097, 5, None) == EALIGN
    assert _rc(L, "utf16_to_well_formed", A, A + 2, 5, None) == EOVERLAP
    assert _rc(L, "utf16_to_well_formed", A + 8, A, 5, None) == EOVERLAP
    assert _rc(L, "utf16_to_well_formed", A, A, 0, None) == 0  # nothing to do
    assert _rc(L, "utf16_to_well_formed_inplace", A + 1, 3, None) == EALIGN
    assert _rc(L, "utf16_is_well_formed", A, 5, None, None) == EINVAL
    assert _rc(L, "utf16_is_well_formed", A, 5, A + 4098, None) == EALIGN
    assert _rc(L, "utf16_is_well_formed", A + 1, 5, A + 4096, None) == EALIGN
    assert _rc(L, "utf16_is_well_formed", A, -2, A + 4096, None) == EINVAL
    assert _rc(L, "utf16_locate_ill_formed", A, 5, A + 4096, A + 4100, None) == EALIGN
    assert _rc(L, "utf16_locate_ill_formed", A, 5, None, A + 4104, None) == EINVAL
    assert _rc(L, "utf16wf_copy_units", A, A + 4098, 4, None) == EALIGN
    msg = L.utf16wf_last_error().decode()
    assert "alignment" in msg or "aligned" in msg


def test_host_path_argument_errors(L):
    import numpy as np
    from paper_2601_06349_amd import EALIGN, EINVAL, EOVERLAP
    s = np.zeros(10, np.uint16)
    p = s.ctypes.data
    assert _rc(L, "utf16_to_well_formed_host", p, p + 2, 10, 0) == EOVERLAP
    assert _rc(L, "utf16_to_well_formed_host", p, p + 1, 10, 0) == EALIGN
    assert _rc(L, "utf16_to_well_formed_host", None, p, 10, 0) == EINVAL
    assert _rc(L, "utf16_to_well_formed_host", p, p, -1, 0) == EINVAL
    assert _rc(L, "utf16_to_well_formed_host", p, p, 10, -5) == EINVAL
    assert _rc(L, "utf16_to_well_formed_host", p, p, 0, 0) == 0


def test_batch_argument_errors(L):
    from paper_2601_06349_amd import EALIGN, EINVAL
    assert _rc(L, "utf16_to_well_formed_batch", A, A + 4096, A + 8192, -1, None) == EINVAL
    assert _rc(L, "utf16_to_well_formed_batch", A, A + 4096, A + 8192, 0, None) == 0
    assert _rc(L, "utf16_to_well_formed_batch", None, A + 4096, A + 8192, 3, None) == EINVAL
    assert _rc(L, "utf16_to_well_formed_batch", A, A + 4096, None, 3, None) == EINVAL
    assert _rc(L, "utf16_to_well_formed_batch", A, A + 4096, A + 8196, 3, None) == EALIGN
    assert _rc(L, "utf16_to_well_formed_batch", A + 1, A + 4096, A + 8192, 3, None) == EALIGN
    assert _rc(L, "utf16_is_well_formed_batch", A, A + 8192, 3, None, None) == EINVAL
    assert _rc(L, "utf16_locate_ill_formed_batch", A, A + 8192, 3, None, A, None) == EINVAL
    assert _rc(L, "utf16wf_batch", 9, A, A, A + 8192, 3, None, None, None, 0, None) == EINVAL
    assert _rc(L, "utf16wf_batch", 1, A, A, A + 8192, 3, None, None, None, -5, None) == EINVAL
    assert _rc(L, "utf16wf_validate_offsets", None, 3, 10, None) == EINVAL
    assert _rc(L, "utf16wf_validate_offsets", A + 4, 3, 10, None) == EALIGN
    assert _rc(L, "utf16wf_validate_offsets", A, -1, 10, None) == EINVAL
    assert _rc(L, "utf16wf_validate_batch", None, A, A + 8192, 3, 10, None) == EINVAL
    assert _rc(L, "utf16wf_validate_batch", A, A + 4096, None, 3, 10, None) == EINVAL
    assert _rc(L, "utf16wf_validate_batch", A + 1, A + 4096, A + 8192, 3, 10, None) == EALIGN
    assert _rc(L, "utf16wf_validate_batch", A, A + 4097, A + 8192, 3, 10, None) == EALIGN
    assert _rc(L, "utf16wf_validate_batch", A, A + 4096, A + 8196, 3, 10, None) == EALIGN
    assert _rc(L, "utf16wf_validate_batch", A, A + 4096, A + 8192, -1, 10, None) == EINVAL


def test_batch_overlap_rejected_with_a_size_hint(L):
    """A batch repair into a distinct buffer spans units_hint units when the
    hint is given: buffers closer than that are rejected before any HIP call
    (in either order, by one unit or by the whole span less one)."""
    from paper_2601_06349_amd import EOVERLAP
    span = 1000
    for d in (2, 100, 2 * span - 2):
        for i, o in ((A, A + d), (A + d, A)):
            assert _rc(L, "utf16wf_batch", 1, i, o, A + 65536, 3, None, None, None, span, None) == EOVERLAP
            assert "overlap" in L.utf16wf_last_error().decode() or "apart" in L.utf16wf_last_error().decode()


class _FakeDeviceTensor:
    """Stands in for a device tensor in the Python wrappers' argument checks,
    which run before any library call (its pointer is never dereferenced)."""

    def __init__(self, dtype, n, device="cuda:0", addr=A):
        import torch
        self.dtype, self._n, self.device, self._addr = dtype, n, torch.device(device), addr
        self.is_cuda = True

    def dim(self):
        return 1

    def is_contiguous(self):
        return True

    def numel(self):
        return self._n

    def data_ptr(self):
        return self._addr


def test_python_batch_wrappers_check_sizes_and_devices():
    import torch
    import paper_2601_06349_amd as wf
    F = _FakeDeviceTensor
    buf, off = F(torch.uint16, 1000), F(torch.int64, 11)  # 10 strings
    with pytest.raises(ValueError, match="fewer than the input"):
        wf.utf16_to_well_formed_batch(buf, off, out=F(torch.uint16, 999))
    with pytest.raises(ValueError, match="fewer than the 10 strings"):
        wf.utf16_is_well_formed_batch(buf, off, results=F(torch.uint8, 9))
    with pytest.raises(TypeError):
        wf.utf16_is_well_formed_batch(buf, off, results=F(torch.int32, 10))
    with pytest.raises(ValueError, match="fewer than the 10 strings"):
        wf.utf16wf_batch(wf.OP_LOCATE, buf, off, first=F(torch.int64, 10), count=F(torch.int64, 3))
    with pytest.raises(ValueError, match="fewer than the 10 strings"):
        wf.utf16wf_batch(wf.OP_IS, buf, off, results=F(torch.uint8, 2))
    with pytest.raises(ValueError, match="fewer than the input"):
        wf.utf16wf_batch(wf.OP_TO, buf, off, out=F(torch.uint16, 10))
    with pytest.raises(ValueError, match="is on"):
        wf.utf16wf_batch(wf.OP_TO, buf, off, out=F(torch.uint16, 1000, device="cuda:1"))
    with pytest.raises(ValueError, match="is on"):
        wf.utf16_to_well_formed_batch(buf, F(torch.int64, 11, device="cuda:1"))
    with pytest.raises(ValueError, match="fewer than the input"):
        wf.BatchPlan(wf.OP_TO, buf, off, out=F(torch.uint16, 5))
    with pytest.raises(ValueError, match="fewer than the 10 strings"):
        wf.BatchPlan(wf.OP_IS, buf, off, results=F(torch.uint8, 1))


def test_plan_argument_errors(L):
    from paper_2601_06349_amd import EINVAL
    h = ctypes.c_void_p()
    assert _rc(L, "utf16wf_batch_plan_create", 1, A, A + 4096, A + 8192, 3, None, None, None) == EINVAL
    assert _rc(L, "utf16wf_batch_plan_create", 7, A, A + 4096, A + 8192, 3, None, None, ctypes.byref(h)) == EINVAL
    assert _rc(L, "utf16wf_batch_plan_create", 3, A, None, A + 8192, 3, None, None, ctypes.byref(h)) == EINVAL
    assert _rc(L, "utf16wf_batch_plan_create", 0, A, None, A + 8192, 3, None, None, ctypes.byref(h)) == EINVAL
    assert _rc(L, "utf16wf_batch_plan_launch", None, None) == EINVAL
    assert _rc(L, "utf16wf_batch_plan_destroy", None) == 0


def test_params_roundtrip(L):
    import paper_2601_06349_amd as wf
    wf.reset_params()
    d = wf.get_params(wf.OP_TO, 0, 1 << 28)
    assert d["rows"] in (1, 2, 4, 8) and 1 <= d["wg_waves"] <= 16
    wf.set_params(wf.OP_TO, 0, 28, rows=8, wg_waves=2, grid_per_cu=3, nontemporal=1)
    assert wf.get_params(wf.OP_TO, 0, (1 << 28) + 5) == {"rows": 8, "wg_waves": 2, "grid_per_cu": 3,
                                                         "nontemporal": 1, "store_lines": 1}
    # the in-place store mode: whole lines by default, changed vectors on request
    assert wf.get_params(wf.OP_TO_INPLACE, 0, 1 << 28)["store_lines"] == 1
    wf.set_params(wf.OP_TO_INPLACE, 0, 28, rows=4, wg_waves=4, grid_per_cu=8, nontemporal=0, store_lines=0)
    assert wf.get_params(wf.OP_TO_INPLACE, 0, 1 << 28)["store_lines"] == 0
    with pytest.raises(wf.Utf16wfError):
        wf.set_params(wf.OP_TO_INPLACE, 0, 28, rows=4, wg_waves=4, grid_per_cu=8, nontemporal=0, store_lines=2)
    assert wf.get_params(wf.OP_TO, 0, 1 << 27) == wf.get_params(wf.OP_TO, 0, (1 << 27) + 1)
    # nearest set class: 2^30 units fall back to class 28
    assert wf.get_params(wf.OP_TO, 0, 1 << 30)["rows"] == 8
    with pytest.raises(wf.Utf16wfError):
        wf.set_params(wf.OP_TO, 0, 28, rows=3, wg_waves=2, grid_per_cu=3, nontemporal=0)
    with pytest.raises(wf.Utf16wfError):
        wf.set_params(wf.OP_TO, 0, 41, rows=4, wg_waves=2, grid_per_cu=3, nontemporal=0)
    with pytest.raises(wf.Utf16wfError):
        wf.set_params(wf.OP_TO, 2, 10, rows=4, wg_waves=2, grid_per_cu=3, nontemporal=0)
    wf.reset_params()
    assert wf.get_params(wf.OP_TO, 0, 1 << 28) == d


def test_product_path_has_no_cpu_route():
    """The package never imports the oracle and the binding has no fallback."""
    pkg = os.path.join(ROOT, "paper_2601_06349_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "utf16_oracle" not in text and "liboracle" not in text, f


def test_tuning_cache_applies(tmp_path, L):
    import json

    import paper_2601_06349_amd as wf
    from paper_2601_06349_amd import tune
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({"entries": [
        {"op": wf.OP_TO, "batch": 0, "size_class": 20,
         "params": {"rows": 2, "wg_waves": 16, "grid_per_cu": 5, "nontemporal": 1}},
        {"op": wf.OP_IS, "batch": 1, "size_class": 40,
         "params": {"rows": 8, "wg_waves": 1, "grid_per_cu": 64, "nontemporal": 0}}]}))
    wf.reset_params()
    try:
        assert tune.apply_cache(str(path)) == "cache.json"
        assert wf.get_params(wf.OP_TO, 0, 1 << 20) == {"rows": 2, "wg_waves": 16, "grid_per_cu": 5,
                                                      "nontemporal": 1, "store_lines": 1}
        assert wf.get_params(wf.OP_IS, 1, 1 << 40)["grid_per_cu"] == 64
        # classes without an entry take the nearest class that has one
        assert wf.get_params(wf.OP_TO, 0, 1 << 21) == wf.get_params(wf.OP_TO, 0, 1 << 20)
        assert wf.get_params(wf.OP_TO, 0, 5) == wf.get_params(wf.OP_TO, 0, 1 << 20)
        assert wf.get_params(wf.OP_IS, 1, 1 << 20)["grid_per_cu"] == 64
        # an (op, batch) with no entry keeps the built-in defaults
        wf.reset_params()
        d = wf.get_params(wf.OP_LOCATE, 1, 1 << 30)
        tune.apply_cache(str(path))
        assert wf.get_params(wf.OP_LOCATE, 1, 1 << 30) == d
    finally:
        wf.reset_params()


def test_committed_tuning_cache_is_valid():
    """Every entry of the committed cache names a valid key and shape."""
    import json
    d = os.path.join(ROOT, "paper_2601_06349_amd", "tuning")
    files = [f for f in os.listdir(d) if f.endswith(".json")]
    assert files
    for f in files:
        data = json.load(open(os.path.join(d, f)))
        for e in data["entries"]:
            p = e["params"]
            assert e["op"] in (0, 1, 2, 3) and e["batch"] in (0, 1) and 0 <= e["size_class"] <= 40
            assert p["rows"] in (1, 2, 4, 8) and 1 <= p["wg_waves"] <= 16 and 1 <= p["grid_per_cu"] <= 64
            assert p.get("store_lines", 1) in (0, 1)
            assert e["tuned_ms"] <= e["default_ms"] * 1.0001
