"""ctypes binding of ``libutf16wf.so`` (the C ABI of include/utf16wf.h).

Argument marshalling only: every step of the check and the repair runs in the
library's HIP kernels. If the library has not been built, loading fails with
an error; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libutf16wf.so")

OK = 0
EINVAL = -1
EALIGN = -2
EOVERLAP = -3
EOFFSETS = -4
EHIP = -5
ERANGE = -6
ENOMEM = -7

OP_IS = 0
OP_TO = 1
OP_TO_INPLACE = 2
OP_LOCATE = 3

_STATUS = {OK: "OK", EINVAL: "EINVAL", EALIGN: "EALIGN", EOVERLAP: "EOVERLAP",
           EOFFSETS: "EOFFSETS", EHIP: "EHIP", ERANGE: "ERANGE", ENOMEM: "ENOMEM"}


class Utf16wfError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_STATUS.get(code, code)}: {message}")
        self.code = code
        self.message = message


class Params(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("wg_waves", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("store_lines", ctypes.c_int32)]

    def __init__(self, rows=0, wg_waves=0, grid_per_cu=0, nontemporal=0, store_lines=1):
        super().__init__(rows, wg_waves, grid_per_cu, nontemporal, store_lines)

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lock = threading.Lock()
_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_INT = ctypes.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "utf16_is_well_formed": (_INT, [_P, _I64, _P, _P]),
    "utf16_to_well_formed": (_INT, [_P, _P, _I64, _P]),
    "utf16_to_well_formed_inplace": (_INT, [_P, _I64, _P]),
    "utf16_locate_ill_formed": (_INT, [_P, _I64, _P, _P, _P]),
    "utf16_to_well_formed_host": (_INT, [_P, _P, _I64, _I64]),
    "utf16_is_well_formed_batch": (_INT, [_P, _P, _I64, _P, _P]),
    "utf16_to_well_formed_batch": (_INT, [_P, _P, _P, _I64, _P]),
    "utf16_to_well_formed_batch_inplace": (_INT, [_P, _P, _I64, _P]),
    "utf16_locate_ill_formed_batch": (_INT, [_P, _P, _I64, _P, _P, _P]),
    "utf16wf_batch": (_INT, [_INT, _P, _P, _P, _I64, _P, _P, _P, _I64, _P]),
    "utf16wf_validate_offsets": (_INT, [_P, _I64, _I64, _P]),
    "utf16wf_validate_batch": (_INT, [_P, _P, _P, _I64, _I64, _P]),
    "utf16wf_validate_batch_noalloc": (_INT, [_P, _P, _P, _I64, _I64, _P]),
    "utf16wf_batch_plan_create": (_INT, [_INT, _P, _P, _P, _I64, _P, _P, ctypes.POINTER(_P)]),
    "utf16wf_batch_plan_launch": (_INT, [_P, _P]),
    "utf16wf_batch_plan_destroy": (_INT, [_P]),
    "utf16wf_set_params": (_INT, [_INT, _INT, _INT, ctypes.POINTER(Params)]),
    "utf16wf_get_params": (_INT, [_INT, _INT, _I64, ctypes.POINTER(Params)]),
    "utf16wf_reset_params": (_INT, []),
    "utf16wf_copy_units": (_INT, [_P, _P, _I64, _P]),
    "utf16wf_device_cus": (_INT, []),
    "utf16wf_serve_run": (_INT, [_P, _P, _I64, _P, _P]),
    "utf16wf_serve_simulate": (_INT, [_P, _P, _P, _I64, _I64, ctypes.c_double, _I64, _P, _P]),
    "utf16wf_last_error": (ctypes.c_char_p, []),
    "utf16wf_abi_version": (_INT, []),
}


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_2601_06349_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return L


def last_error() -> str:
    return (lib().utf16wf_last_error() or b"").decode(errors="replace")


def check(rc: int) -> int:
    if rc != OK:
        raise Utf16wfError(rc, last_error())
    return rc
