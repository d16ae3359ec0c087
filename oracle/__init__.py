"""CPU oracle for UTF-16 well-formedness repair (ctypes front-end).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users. The product library never imports, links
or calls anything under ``oracle/``, and this package imports nothing from the
product package.

The arithmetic lives in ``utf16_oracle.c`` (plain scalar C, built with
``-O2 -fno-tree-vectorize``). It is the sequential definition from
Clausecker & Lemire, arXiv 2601.06349: Sec. 1 (surrogate ranges, the
ill-formedness definition), the Abstract and Sec. 3.1 (one U+FFFD per
mismatched unit, length kept), Sec. 3.1 edge cases (a leading low and a
trailing high are mismatched). Ragged batches repair each string alone.

Parity pins for every function here are in ``tests/test_oracle_pins.py``;
``wf_locate_batch`` (first bad index and count per string) is pinned there by
brute force and by the Python codec.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "utf16_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_utf16.so")

_lib = None


def build() -> str:
    """Compile the oracle shared library with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fno-tree-vectorize", "-fPIC", "-shared",
           "-pthread", "-Wall", "-Wextra", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib_path() -> str:
    """The oracle library to load: the build named by UTF16WF_ORACLE_LIB if
    set (the sanitizer test builds utf16_oracle.c with AddressSanitizer and
    UBSan), else the plain build, compiled first if missing or stale."""
    path = os.environ.get("UTF16WF_ORACLE_LIB")
    if path:
        return path
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(lib_path())
    p16 = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.wf_to_seq.argtypes = [p16, p16, i64]
    lib.wf_to_seq.restype = i64
    lib.wf_is_seq.argtypes = [p16, i64]
    lib.wf_is_seq.restype = ctypes.c_int
    lib.wf_first_bad_seq.argtypes = [p16, i64]
    lib.wf_first_bad_seq.restype = i64
    lib.wf_to_batch.argtypes = [p16, p16, p16, i64]
    lib.wf_to_batch.restype = i64
    lib.wf_is_batch.argtypes = [p16, p16, i64, p16]
    lib.wf_is_batch.restype = None
    lib.wf_locate_batch.argtypes = [p16, p16, i64, p16, p16]
    lib.wf_locate_batch.restype = None
    lib.wf_to_chunked_mt.argtypes = [p16, p16, i64, ctypes.c_int]
    lib.wf_to_chunked_mt.restype = i64
    _lib = lib
    return lib


def _u16(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype != np.uint16:
        a = a.astype(np.uint16)
    return np.ascontiguousarray(a)


def _offs(off) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(off, dtype=np.int64))


def to_well_formed(s) -> np.ndarray:
    """Repaired copy of ``s`` (uint16 array)."""
    s = _u16(s)
    t = np.empty_like(s)
    _load().wf_to_seq(s.ctypes.data, t.ctypes.data, s.size)
    return t


def to_well_formed_count(s):
    """(repaired copy, number of units replaced)."""
    s = _u16(s)
    t = np.empty_like(s)
    c = _load().wf_to_seq(s.ctypes.data, t.ctypes.data, s.size)
    return t, int(c)


def is_well_formed(s) -> bool:
    s = _u16(s)
    return bool(_load().wf_is_seq(s.ctypes.data, s.size))


def first_bad(s) -> int:
    s = _u16(s)
    return int(_load().wf_first_bad_seq(s.ctypes.data, s.size))


def to_well_formed_batch(buf, offsets, out=None) -> np.ndarray:
    """Per-string repair of a packed buffer. Units outside [off[0], off[B])
    keep the values of ``out`` (a copy of ``buf`` when ``out`` is None)."""
    buf = _u16(buf)
    off = _offs(offsets)
    t = buf.copy() if out is None else _u16(out).copy()
    _load().wf_to_batch(buf.ctypes.data, t.ctypes.data, off.ctypes.data, off.size - 1)
    return t


def is_well_formed_batch(buf, offsets) -> np.ndarray:
    buf = _u16(buf)
    off = _offs(offsets)
    res = np.empty(off.size - 1, dtype=np.uint8)
    _load().wf_is_batch(buf.ctypes.data, off.ctypes.data, off.size - 1, res.ctypes.data)
    return res


def locate_batch(buf, offsets):
    """(first_bad[k] relative to the string start or -1, count[k])."""
    buf = _u16(buf)
    off = _offs(offsets)
    b = off.size - 1
    first = np.empty(b, dtype=np.int64)
    cnt = np.empty(b, dtype=np.int64)
    _load().wf_locate_batch(buf.ctypes.data, off.ctypes.data, b, first.ctypes.data, cnt.ctypes.data)
    return first, cnt


def to_well_formed_mt(s, threads: int | None = None) -> np.ndarray:
    """Chunked multi-threaded repair (same result as ``to_well_formed``)."""
    s = _u16(s)
    t = np.empty_like(s)
    th = threads or os.cpu_count() or 1
    r = _load().wf_to_chunked_mt(s.ctypes.data, t.ctypes.data, s.size, int(th))
    if r < 0:
        raise RuntimeError("oracle: thread creation failed")
    return t
