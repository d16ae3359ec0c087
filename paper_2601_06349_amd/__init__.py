"""UTF-16 well-formedness check and repair on MI355X (gfx950).

Python front-end of ``libutf16wf.so``. PyTorch supplies device memory and
streams; every step of the check and the repair runs in the library's HIP
kernels (the functions below only marshal pointers, sizes and the stream).

Tensors of code units are 1-D, contiguous, on a CUDA (HIP) device, with dtype
``torch.uint16`` or ``torch.int16`` (the same 16 bits). Offsets are
contiguous ``torch.int64`` on the same device. Calls run on the current torch
stream unless ``stream`` is given.

The operation is the one of Clausecker & Lemire, arXiv 2601.06349 (Sec. 1 and
Sec. 3.1): every high surrogate not followed by a low one and every low
surrogate not preceded by a high one is replaced with U+FFFD; the length is
kept; a leading low and a trailing high are mismatched. Ragged batches treat
each string alone.
"""
from __future__ import annotations

import ctypes

from ._lib import (EALIGN, EHIP, EINVAL, ENOMEM, EOFFSETS, EOVERLAP, ERANGE, OK, OP_IS, OP_LOCATE, OP_TO,
                   OP_TO_INPLACE, Params, Utf16wfError, check, last_error, lib)

__all__ = [
    "utf16_is_well_formed", "utf16_to_well_formed", "utf16_to_well_formed_inplace",
    "utf16_locate_ill_formed", "utf16_to_well_formed_host", "utf16_is_well_formed_batch", "utf16_to_well_formed_batch",
    "utf16_to_well_formed_batch_inplace", "utf16_locate_ill_formed_batch", "utf16wf_batch",
    "utf16wf_validate_offsets", "utf16wf_validate_batch", "BatchPlan", "is_well_formed", "set_params", "get_params",
    "reset_params", "utf16wf_copy_units", "device_cus", "Utf16wfError", "lib", "last_error",
    "OP_IS", "OP_TO", "OP_TO_INPLACE", "OP_LOCATE", "OK", "EINVAL", "EALIGN", "EOVERLAP",
    "EOFFSETS", "EHIP", "ERANGE", "ENOMEM",
]


def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _units(t, name="input"):
    torch = _torch()
    if t.dtype not in (torch.uint16, torch.int16):
        raise TypeError(f"{name} must be torch.uint16 or torch.int16, got {t.dtype}")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be 1-D and contiguous")
    return t


def _offsets(off):
    torch = _torch()
    if off.dtype != torch.int64 or not off.is_cuda or off.dim() != 1 or not off.is_contiguous():
        raise TypeError("offsets must be a contiguous 1-D torch.int64 device tensor")
    if off.numel() < 1:
        raise ValueError("offsets needs num_strings + 1 entries")
    return off


def _same_device(name, t, ref):
    if t.device != ref.device:
        raise ValueError(f"{name} is on {t.device}, the input on {ref.device}")


def _batch_out(out, buf):
    """A caller's output buffer of a batch repair: code units on the input's
    device, with room for every unit the offsets may name (those of buf)."""
    _units(out, "out")
    _same_device("out", out, buf)
    if out.numel() < buf.numel():
        raise ValueError(f"out has {out.numel()} units, fewer than the input's {buf.numel()}")
    return out


def _per_string(name, t, dtype, b, buf):
    """A caller's per-string result array: at least b entries of dtype,
    contiguous, on the input's device."""
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} device tensor")
    _same_device(name, t, buf)
    if t.numel() < b:
        raise ValueError(f"{name} has {t.numel()} entries, fewer than the {b} strings")
    return t


def utf16_is_well_formed(t, result=None, stream=None):
    """Device int32 tensor [1]: 1 if ``t`` is well-formed, else 0."""
    torch = _torch()
    _units(t)
    if result is None:
        result = torch.empty(1, dtype=torch.int32, device=t.device)
    check(lib().utf16_is_well_formed(t.data_ptr(), t.numel(), result.data_ptr(), _stream(stream)))
    return result


def is_well_formed(t, stream=None) -> bool:
    """Synchronising convenience: ``bool`` result of isWellFormed."""
    return bool(utf16_is_well_formed(t, stream=stream).item())


def utf16_to_well_formed(t, out=None, stream=None):
    """Repaired copy of ``t`` (``out`` may be ``t`` for in place)."""
    torch = _torch()
    _units(t)
    if out is None:
        out = torch.empty_like(t)
    _units(out, "out")
    if out.numel() != t.numel():
        raise ValueError("out must have as many units as the input")
    check(lib().utf16_to_well_formed(t.data_ptr(), out.data_ptr(), t.numel(), _stream(stream)))
    return out


def utf16_to_well_formed_inplace(t, stream=None):
    _units(t)
    check(lib().utf16_to_well_formed_inplace(t.data_ptr(), t.numel(), _stream(stream)))
    return t


def utf16_to_well_formed_host(arr, out=None, chunk_units=0):
    """Repair a host-resident numpy uint16 array (``out`` may be ``arr`` for
    in place) through device staging in overlapped chunks; returns ``out``.
    Pinned host memory (e.g. the numpy view of a torch ``pin_memory``
    tensor) lets copies and repairs overlap."""
    import numpy as np
    if not isinstance(arr, np.ndarray) or arr.dtype not in (np.uint16, np.int16) or arr.ndim != 1 \
            or not arr.flags.c_contiguous:
        raise TypeError("arr must be a contiguous 1-D numpy uint16 array")
    if out is None:
        out = np.empty_like(arr)
    if out.shape != arr.shape or out.dtype != arr.dtype or not out.flags.c_contiguous:
        raise ValueError("out must match arr")
    check(lib().utf16_to_well_formed_host(arr.ctypes.data, out.ctypes.data, arr.size, int(chunk_units)))
    return out


def utf16_locate_ill_formed(t, stream=None):
    """Device int64 tensor [2]: (index of the first mismatched unit or -1,
    number of mismatched units)."""
    torch = _torch()
    _units(t)
    res = torch.empty(2, dtype=torch.int64, device=t.device)
    check(lib().utf16_locate_ill_formed(t.data_ptr(), t.numel(), res.data_ptr(), res.data_ptr() + 8,
                                        _stream(stream)))
    return res


def utf16_is_well_formed_batch(buf, offsets, results=None, stream=None):
    """Device uint8 tensor [B]: 1 where string k is well-formed."""
    torch = _torch()
    _units(buf)
    _offsets(offsets)
    _same_device("offsets", offsets, buf)
    b = offsets.numel() - 1
    if results is None:
        results = torch.empty(b, dtype=torch.uint8, device=buf.device)
    _per_string("results", results, torch.uint8, b, buf)
    check(lib().utf16_is_well_formed_batch(buf.data_ptr(), offsets.data_ptr(), b, results.data_ptr(),
                                           _stream(stream)))
    return results


def utf16_to_well_formed_batch(buf, offsets, out=None, stream=None):
    """Per-string repair. Units of ``out`` outside [off[0], off[B]) are not
    written (a fresh ``out`` starts as a copy of ``buf``)."""
    _units(buf)
    _offsets(offsets)
    _same_device("offsets", offsets, buf)
    if out is None:
        out = buf.clone()
    _batch_out(out, buf)
    check(lib().utf16_to_well_formed_batch(buf.data_ptr(), out.data_ptr(), offsets.data_ptr(),
                                           offsets.numel() - 1, _stream(stream)))
    return out


def utf16_to_well_formed_batch_inplace(buf, offsets, stream=None):
    _units(buf)
    _offsets(offsets)
    _same_device("offsets", offsets, buf)
    check(lib().utf16_to_well_formed_batch_inplace(buf.data_ptr(), offsets.data_ptr(), offsets.numel() - 1,
                                                   _stream(stream)))
    return buf


def utf16_locate_ill_formed_batch(buf, offsets, stream=None):
    """(first_bad, count) device int64 tensors [B]; first_bad is relative to
    the string start, -1 when the string is well-formed."""
    torch = _torch()
    _units(buf)
    _offsets(offsets)
    _same_device("offsets", offsets, buf)
    b = offsets.numel() - 1
    first = torch.empty(b, dtype=torch.int64, device=buf.device)
    count = torch.empty(b, dtype=torch.int64, device=buf.device)
    check(lib().utf16_locate_ill_formed_batch(buf.data_ptr(), offsets.data_ptr(), b, first.data_ptr(),
                                              count.data_ptr(), _stream(stream)))
    return first, count


def utf16wf_batch(op, buf, offsets, out=None, results=None, first=None, count=None, units_hint=0, stream=None):
    """General batch entry (see the C header)."""
    _check_batch_buffers(op, buf, offsets, out, results, first, count)
    ptr = (lambda x: x.data_ptr() if x is not None else None)
    check(lib().utf16wf_batch(int(op), buf.data_ptr(), ptr(out), offsets.data_ptr(), offsets.numel() - 1,
                              ptr(results), ptr(first), ptr(count), int(units_hint), _stream(stream)))


def _check_batch_buffers(op, buf, offsets, out=None, results=None, first=None, count=None):
    """Every buffer a batch call of `op` writes is on the input's device and
    large enough for the strings the offsets name."""
    torch = _torch()
    _units(buf)
    _offsets(offsets)
    _same_device("offsets", offsets, buf)
    b = offsets.numel() - 1
    if out is not None:
        _batch_out(out, buf)
    if op == OP_IS and results is not None:
        _per_string("results", results, torch.uint8, b, buf)
    if op == OP_LOCATE:
        for name, t in (("first", first), ("count", count)):
            if t is not None:
                _per_string(name, t, torch.int64, b, buf)


def utf16wf_validate_batch(buf, offsets, out=None, stream=None):
    """Raises Utf16wfError(EOFFSETS) unless the offsets are non-decreasing
    within [0, buf.numel()], and Utf16wfError(EOVERLAP) when ``out`` (neither
    None nor ``buf``) overlaps ``buf`` over the units the batch spans.
    Synchronises the stream."""
    _units(buf)
    _offsets(offsets)
    if out is not None:
        _units(out, "out")
    check(lib().utf16wf_validate_batch(buf.data_ptr(), out.data_ptr() if out is not None else None,
                                       offsets.data_ptr(), offsets.numel() - 1, buf.numel(), _stream(stream)))


def utf16wf_validate_offsets(offsets, buf_units, stream=None):
    """Raises Utf16wfError(EOFFSETS) unless offsets are non-decreasing within
    [0, buf_units]. Synchronises the stream."""
    _offsets(offsets)
    check(lib().utf16wf_validate_offsets(offsets.data_ptr(), offsets.numel() - 1, int(buf_units), _stream(stream)))


class BatchPlan:
    """A batch call captured once into a HIP graph and replayed by launch()."""

    def __init__(self, op, buf, offsets, out=None, results=None, stream=None):
        _check_batch_buffers(op, buf, offsets, out, results)
        self._keep = (buf, offsets, out, results)  # keep the buffers alive
        h = ctypes.c_void_p()
        check(lib().utf16wf_batch_plan_create(
            int(op), buf.data_ptr(), out.data_ptr() if out is not None else None, offsets.data_ptr(),
            offsets.numel() - 1, results.data_ptr() if results is not None else None, _stream(stream),
            ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        check(lib().utf16wf_batch_plan_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().utf16wf_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_params(op, batch, size_class, rows, wg_waves, grid_per_cu, nontemporal, store_lines=1):
    p = Params(rows, wg_waves, grid_per_cu, nontemporal, store_lines)
    check(lib().utf16wf_set_params(int(op), int(batch), int(size_class), ctypes.byref(p)))


def get_params(op, batch, n) -> dict:
    p = Params()
    check(lib().utf16wf_get_params(int(op), int(batch), int(n), ctypes.byref(p)))
    return p.as_dict()


def reset_params():
    check(lib().utf16wf_reset_params())


def utf16wf_copy_units(src, dst, stream=None):
    _units(src)
    _units(dst, "dst")
    check(lib().utf16wf_copy_units(src.data_ptr(), dst.data_ptr(), src.numel(), _stream(stream)))
    return dst


def device_cus() -> int:
    return int(lib().utf16wf_device_cus())
