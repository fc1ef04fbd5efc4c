"""Python binding of the scalar CPU oracle (``oracle/utf_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference that the
GPU library is checked against.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark import this module; the GPU library never
does, and the two share no code.

Every function takes numpy arrays living in host memory:

* UTF-8 text is a ``uint8`` array.
* UTF-16LE text is a ``uint16`` array (little-endian words); it is handed to
  the C code as its raw bytes, which the oracle reassembles low byte first.

Results mirror the GPU library's convention: ``(status, count)`` where
``status == 0`` means OK and ``count`` is the number of units validated or
written, ``1..8`` are data errors with ``count`` the first-error offset in
input units, and ``9`` (OUTPUT_TOO_SMALL) carries the number of units needed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "utf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# The oracle's own copy of the status convention.
OK = 0
TOO_SHORT = 1
TOO_LONG = 2
OVERLONG = 3
TOO_LARGE = 4
SURROGATE = 5
HEADER_BITS = 6
UNPAIRED_HIGH = 7
UNPAIRED_LOW = 8
OUTPUT_TOO_SMALL = 9

STATUS_NAMES = {
    OK: "OK", TOO_SHORT: "TOO_SHORT", TOO_LONG: "TOO_LONG",
    OVERLONG: "OVERLONG", TOO_LARGE: "TOO_LARGE", SURROGATE: "SURROGATE",
    HEADER_BITS: "HEADER_BITS", UNPAIRED_HIGH: "UNPAIRED_HIGH",
    UNPAIRED_LOW: "UNPAIRED_LOW", OUTPUT_TOO_SMALL: "OUTPUT_TOO_SMALL",
}


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("count", ctypes.c_uint64)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra",
                               "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    P = ctypes.c_void_p
    U64 = ctypes.c_uint64
    for name in ("oracle_validate_utf8", "oracle_validate_utf16le"):
        f = getattr(lib, name)
        f.argtypes = [P, U64]
        f.restype = _Result
    for name in ("oracle_utf16_length_from_utf8", "oracle_utf8_length_from_utf16le"):
        f = getattr(lib, name)
        f.argtypes = [P, U64]
        f.restype = U64
    for name in ("oracle_convert_utf8_to_utf16le", "oracle_convert_utf16le_to_utf8"):
        f = getattr(lib, name)
        f.argtypes = [P, U64, P, U64]
        f.restype = _Result
    for name in ("oracle_validate_utf8_batch", "oracle_validate_utf16le_batch"):
        f = getattr(lib, name)
        f.argtypes = [P, P, U64, P]
        f.restype = None
    for name in ("oracle_convert_utf8_to_utf16le_batch", "oracle_convert_utf16le_to_utf8_batch"):
        f = getattr(lib, name)
        f.argtypes = [P, P, U64, P, P, P]
        f.restype = None
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def _u8(a) -> np.ndarray:
    a = np.ascontiguousarray(np.frombuffer(a, dtype=np.uint8) if isinstance(a, (bytes, bytearray)) else a)
    assert a.dtype == np.uint8, a.dtype
    return a


def _u16(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray)):
        assert len(a) % 2 == 0
        a = np.frombuffer(a, dtype="<u2")
    a = np.ascontiguousarray(a)
    assert a.dtype == np.uint16, a.dtype
    return a


def validate_utf8(s, lib=None) -> Tuple[int, int]:
    s = _u8(s)
    r = (lib or load()).oracle_validate_utf8(_ptr(s), s.size)
    return r.status, r.count


def validate_utf16le(s, lib=None) -> Tuple[int, int]:
    s = _u16(s)
    r = (lib or load()).oracle_validate_utf16le(_ptr(s), s.size)
    return r.status, r.count


def utf16_length_from_utf8(s, lib=None) -> int:
    s = _u8(s)
    return int((lib or load()).oracle_utf16_length_from_utf8(_ptr(s), s.size))


def utf8_length_from_utf16le(s, lib=None) -> int:
    s = _u16(s)
    return int((lib or load()).oracle_utf8_length_from_utf16le(_ptr(s), s.size))


def convert_utf8_to_utf16le(s, cap: int | None = None, lib=None):
    """Returns ``(status, count, out)``; ``out`` is a uint16 array of ``cap`` words."""
    s = _u8(s)
    if cap is None:
        cap = s.size
    out = np.zeros(cap, dtype=np.uint16)
    r = (lib or load()).oracle_convert_utf8_to_utf16le(_ptr(s), s.size, _ptr(out), cap)
    return r.status, r.count, out


def convert_utf16le_to_utf8(s, cap: int | None = None, lib=None):
    """Returns ``(status, count, out)``; ``out`` is a uint8 array of ``cap`` bytes."""
    s = _u16(s)
    if cap is None:
        cap = 3 * s.size
    out = np.zeros(cap, dtype=np.uint8)
    r = (lib or load()).oracle_convert_utf16le_to_utf8(_ptr(s), s.size, _ptr(out), cap)
    return r.status, r.count, out


def _results_to_arrays(res) -> Tuple[np.ndarray, np.ndarray]:
    raw = np.frombuffer(res, dtype=np.dtype([("status", "<i4"), ("pad", "<i4"), ("count", "<u8")]))
    return raw["status"].copy(), raw["count"].copy()


def validate_utf8_batch(s, offsets, lib=None):
    s = _u8(s)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = offsets.size - 1
    res = (_Result * max(k, 1))()
    (lib or load()).oracle_validate_utf8_batch(_ptr(s), _ptr(offsets), k, ctypes.addressof(res))
    st, cnt = _results_to_arrays(res)
    return st[:k], cnt[:k]


def validate_utf16le_batch(s, offsets, lib=None):
    s = _u16(s)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = offsets.size - 1
    res = (_Result * max(k, 1))()
    (lib or load()).oracle_validate_utf16le_batch(_ptr(s), _ptr(offsets), k, ctypes.addressof(res))
    st, cnt = _results_to_arrays(res)
    return st[:k], cnt[:k]


def convert_utf8_to_utf16le_batch(s, offsets, lib=None):
    """Returns ``(status[k], count[k], out uint16[total], out_offsets int64[k+1])``."""
    s = _u8(s)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = offsets.size - 1
    total = utf16_length_from_utf8(s[offsets[0]:offsets[-1]], lib=lib) if k > 0 else 0
    out = np.zeros(max(total, 1), dtype=np.uint16)
    out_offsets = np.zeros(k + 1, dtype=np.int64)
    res = (_Result * max(k, 1))()
    (lib or load()).oracle_convert_utf8_to_utf16le_batch(
        _ptr(s), _ptr(offsets), k, _ptr(out), _ptr(out_offsets), ctypes.addressof(res))
    st, cnt = _results_to_arrays(res)
    return st[:k], cnt[:k], out[:total], out_offsets


def convert_utf16le_to_utf8_batch(s, offsets, lib=None):
    """Returns ``(status[k], count[k], out uint8[total], out_offsets int64[k+1])``."""
    s = _u16(s)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = offsets.size - 1
    total = utf8_length_from_utf16le(s[offsets[0]:offsets[-1]], lib=lib) if k > 0 else 0
    out = np.zeros(max(total, 1), dtype=np.uint8)
    out_offsets = np.zeros(k + 1, dtype=np.int64)
    res = (_Result * max(k, 1))()
    (lib or load()).oracle_convert_utf16le_to_utf8_batch(
        _ptr(s), _ptr(offsets), k, _ptr(out), _ptr(out_offsets), ctypes.addressof(res))
    st, cnt = _results_to_arrays(res)
    return st[:k], cnt[:k], out[:total], out_offsets
