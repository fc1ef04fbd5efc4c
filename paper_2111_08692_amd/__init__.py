"""Python binding of ``libutfgpu.so``, the gfx950 UTF-8 <-> UTF-16LE library.

Argument marshalling only: every step of validation, length computation and
conversion runs in the library's HIP kernels.  PyTorch supplies device
memory (tensors on ``cuda``) and streams.  The functions carry the names of
the C ABI in ``include/utfgpu.h``:

* ``validate_utf8(t)`` / ``validate_utf16le(t)`` -> ``(status, count)``
* ``utf16_length_from_utf8(t)`` / ``utf8_length_from_utf16le(t)`` -> int
* ``convert_utf8_to_utf16le(t, out=None)`` -> ``(status, count, out)``
* ``convert_utf16le_to_utf8(t, out=None)`` -> ``(status, count, out)``
* ``convert_utf8_to_utf16le_batch_async(t, offsets, out, out_offsets, results)``
  (k strings back to back, one call)

UTF-8 tensors are ``torch.uint8``; UTF-16LE tensors have 2-byte elements
(``torch.int16`` by default: the library only reads the bytes).  All must be contiguous CUDA (HIP) tensors.  The
library is loaded from this directory on first use and every call raises
if it was not built, so no call can silently fall back to another
implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libutfgpu.so")

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
ERR_NULL = -1
ERR_ALIGN = -2
ERR_TOO_BIG = -3
ERR_HIP = -4
ERR_OFFSETS = -5
ERR_ARG = -6

# operations of the geometry tuning table
OP_VALIDATE_UTF8 = 0
OP_CONVERT_UTF8 = 1
OP_VALIDATE_UTF16LE = 2
OP_CONVERT_UTF16LE = 3
OP_BATCH_UTF8 = 4
OP_BATCH_UTF16LE = 5
OP_COUNT = 6
SIZE_CLASSES = 64

# scan schedules (order in which workgroups take tiles)
SCHEDULE_BLOCK = 0
SCHEDULE_TICKET = 1
SCHEDULE_NAMES = ("block", "ticket")

STATUS_NAMES = {
    OK: "OK", TOO_SHORT: "TOO_SHORT", TOO_LONG: "TOO_LONG", OVERLONG: "OVERLONG",
    TOO_LARGE: "TOO_LARGE", SURROGATE: "SURROGATE", HEADER_BITS: "HEADER_BITS",
    UNPAIRED_HIGH: "UNPAIRED_HIGH", UNPAIRED_LOW: "UNPAIRED_LOW",
    OUTPUT_TOO_SMALL: "OUTPUT_TOO_SMALL", ERR_NULL: "ERR_NULL", ERR_ALIGN: "ERR_ALIGN",
    ERR_TOO_BIG: "ERR_TOO_BIG", ERR_HIP: "ERR_HIP", ERR_OFFSETS: "ERR_OFFSETS", ERR_ARG: "ERR_ARG",
}

EXPORTS = (
    "validate_utf8", "validate_utf16le", "utf16_length_from_utf8", "utf8_length_from_utf16le",
    "convert_utf8_to_utf16le", "convert_utf16le_to_utf8",
    "validate_utf8_async", "validate_utf16le_async", "utf16_length_from_utf8_async",
    "utf8_length_from_utf16le_async", "convert_utf8_to_utf16le_async",
    "convert_utf16le_to_utf8_async", "convert_utf8_to_utf16le_batch_async", "convert_utf16le_to_utf8_batch_async",
    "utfgpu_release_workspace", "utfgpu_version", "utfgpu_tile_bytes",
    "utfgpu_geometry_count", "utfgpu_geometry", "utfgpu_set_geometry", "utfgpu_get_geometry", "utfgpu_size_class",
    "utfgpu_set_schedule", "utfgpu_get_schedule",
    "convert_utf8_to_utf16le_noalloc_async",
)


class UtfResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("count", ctypes.c_uint64)]


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    P, U64, I32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32
    sig = {
        "validate_utf8": ([P, U64, P], UtfResult),
        "validate_utf16le": ([P, U64, P], UtfResult),
        "utf16_length_from_utf8": ([P, U64, P], U64),
        "utf8_length_from_utf16le": ([P, U64, P], U64),
        "convert_utf8_to_utf16le": ([P, U64, P, U64, P], UtfResult),
        "convert_utf16le_to_utf8": ([P, U64, P, U64, P], UtfResult),
        "validate_utf8_async": ([P, U64, P, P], I32),
        "validate_utf16le_async": ([P, U64, P, P], I32),
        "utf16_length_from_utf8_async": ([P, U64, P, P], I32),
        "utf8_length_from_utf16le_async": ([P, U64, P, P], I32),
        "convert_utf8_to_utf16le_async": ([P, U64, P, U64, P, P], I32),
        "convert_utf16le_to_utf8_async": ([P, U64, P, U64, P, P], I32),
        "convert_utf8_to_utf16le_batch_async": ([P, U64, P, U64, P, U64, P, P, P], I32),
        "convert_utf16le_to_utf8_batch_async": ([P, U64, P, U64, P, U64, P, P, P], I32),
        "utfgpu_release_workspace": ([], I32),
        "utfgpu_version": ([], ctypes.c_char_p),
        "utfgpu_tile_bytes": ([], U64),
        "utfgpu_geometry_count": ([], I32),
        "utfgpu_geometry": ([I32, P, P, P], I32),
        "utfgpu_set_geometry": ([I32, I32, I32], I32),
        "utfgpu_get_geometry": ([I32, I32], I32),
        "utfgpu_size_class": ([U64], I32),
        "utfgpu_set_schedule": ([I32, I32, I32], I32),
        "utfgpu_get_schedule": ([I32, I32], I32),
        "convert_utf8_to_utf16le_noalloc_async": ([P, U64, P, U64, P, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with paper_2111_08692_amd.build.build() "
            "(hipcc --offload-arch=gfx950); there is no other implementation")
    return _declare(ctypes.CDLL(LIB_PATH))


_lib: Optional[ctypes.CDLL] = None


def load() -> ctypes.CDLL:
    """The loaded library (loads it on first use; raises if it is not built)."""
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def version() -> str:
    return load().utfgpu_version().decode()


def tile_bytes() -> int:
    """Input bytes one workgroup of the validate/convert kernels covers."""
    return int(load().utfgpu_tile_bytes())


def release_workspace() -> int:
    return int(load().utfgpu_release_workspace())


def geometries() -> list:
    """``(waves, rows, tile_bytes)`` of every compiled tile geometry (index 0
    is the default)."""
    lib = load()
    out = []
    for g in range(int(lib.utfgpu_geometry_count())):
        w, r, tb = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        rc = lib.utfgpu_geometry(g, ctypes.byref(w), ctypes.byref(r), ctypes.byref(tb))
        if rc != OK:
            raise RuntimeError(f"utfgpu_geometry({g}) failed: {rc}")
        out.append((int(w.value), int(r.value), int(tb.value)))
    return out


def set_geometry(op: int, size_class: int, g: int) -> int:
    """Calls of ``op`` whose input falls in ``size_class`` use geometry ``g``
    (-1: the default).  Returns the C status."""
    return int(load().utfgpu_set_geometry(int(op), int(size_class), int(g)))


def get_geometry(op: int, size_class: int) -> int:
    return int(load().utfgpu_get_geometry(int(op), int(size_class)))


def set_schedule(op: int, size_class: int, schedule: int) -> int:
    """Calls of ``op`` whose input falls in ``size_class`` use scan schedule
    ``schedule`` (SCHEDULE_BLOCK or SCHEDULE_TICKET; -1: the default).
    Returns the C status."""
    return int(load().utfgpu_set_schedule(int(op), int(size_class), int(schedule)))


def get_schedule(op: int, size_class: int) -> int:
    return int(load().utfgpu_get_schedule(int(op), int(size_class)))


def size_class(nbytes: int) -> int:
    """The tuning-table size class of an input of ``nbytes`` bytes."""
    return int(load().utfgpu_size_class(int(nbytes)))


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev(t: torch.Tensor, elem: int, what: str) -> None:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.element_size() != elem:
        raise ValueError(f"{what} must have {elem}-byte elements")


def _ptr(t: Optional[torch.Tensor]) -> int:
    return 0 if t is None or t.numel() == 0 else t.data_ptr()


# ---------------------------------------------------------------------------
# the C ABI, one function each
# ---------------------------------------------------------------------------

def validate_utf8(data: torch.Tensor, stream=None) -> Tuple[int, int]:
    _dev(data, 1, "data")
    r = load().validate_utf8(_ptr(data), data.numel(), _stream(stream))
    return r.status, r.count


def validate_utf16le(data: torch.Tensor, stream=None) -> Tuple[int, int]:
    _dev(data, 2, "data")
    r = load().validate_utf16le(_ptr(data), data.numel(), _stream(stream))
    return r.status, r.count


def utf16_length_from_utf8(data: torch.Tensor, stream=None) -> int:
    _dev(data, 1, "data")
    return int(load().utf16_length_from_utf8(_ptr(data), data.numel(), _stream(stream)))


def utf8_length_from_utf16le(data: torch.Tensor, stream=None) -> int:
    _dev(data, 2, "data")
    return int(load().utf8_length_from_utf16le(_ptr(data), data.numel(), _stream(stream)))


def convert_utf8_to_utf16le(data: torch.Tensor, out: Optional[torch.Tensor] = None,
                            out_cap: Optional[int] = None, stream=None):
    """Returns ``(status, count, out)``; ``out`` defaults to ``data.numel()``
    words (int16 storage)."""
    _dev(data, 1, "data")
    if out is None:
        out = torch.empty(max(data.numel(), 1), dtype=torch.int16, device=data.device)
    _dev(out, 2, "out")
    cap = out.numel() if out_cap is None else int(out_cap)
    r = load().convert_utf8_to_utf16le(_ptr(data), data.numel(), _ptr(out), cap, _stream(stream))
    return r.status, r.count, out


def convert_utf16le_to_utf8(data: torch.Tensor, out: Optional[torch.Tensor] = None,
                            out_cap: Optional[int] = None, stream=None):
    """Returns ``(status, count, out)``; ``out`` defaults to ``3 * data.numel()`` bytes."""
    _dev(data, 2, "data")
    if out is None:
        out = torch.empty(max(3 * data.numel(), 1), dtype=torch.uint8, device=data.device)
    _dev(out, 1, "out")
    cap = out.numel() if out_cap is None else int(out_cap)
    r = load().convert_utf16le_to_utf8(_ptr(data), data.numel(), _ptr(out), cap, _stream(stream))
    return r.status, r.count, out


# asynchronous forms: results land in device tensors (int64[2] per utf_result)

def result_tensor(device="cuda") -> torch.Tensor:
    """Device storage for one ``utf_result`` (status in the low word of [0])."""
    return torch.zeros(2, dtype=torch.int64, device=device)


def decode_result(t: torch.Tensor) -> Tuple[int, int]:
    v = t.cpu().tolist()
    status = v[0] & 0xFFFFFFFF
    if status >= 1 << 31:
        status -= 1 << 32
    return status, v[1] & 0xFFFFFFFFFFFFFFFF


def validate_utf8_async(data, result, stream=None) -> int:
    _dev(data, 1, "data")
    return int(load().validate_utf8_async(_ptr(data), data.numel(), result.data_ptr(), _stream(stream)))


def validate_utf16le_async(data, result, stream=None) -> int:
    _dev(data, 2, "data")
    return int(load().validate_utf16le_async(_ptr(data), data.numel(), result.data_ptr(), _stream(stream)))


def utf16_length_from_utf8_async(data, result, stream=None) -> int:
    _dev(data, 1, "data")
    return int(load().utf16_length_from_utf8_async(_ptr(data), data.numel(), result.data_ptr(), _stream(stream)))


def utf8_length_from_utf16le_async(data, result, stream=None) -> int:
    _dev(data, 2, "data")
    return int(load().utf8_length_from_utf16le_async(_ptr(data), data.numel(), result.data_ptr(), _stream(stream)))


def convert_utf8_to_utf16le_async(data, out, result, out_cap=None, stream=None) -> int:
    _dev(data, 1, "data")
    _dev(out, 2, "out")
    cap = out.numel() if out_cap is None else int(out_cap)
    return int(load().convert_utf8_to_utf16le_async(_ptr(data), data.numel(), _ptr(out), cap,
                                                 result.data_ptr(), _stream(stream)))


def convert_utf8_to_utf16le_noalloc_async(data, out, result, out_cap=None, stream=None) -> int:
    """The allocation-free form of ``convert_utf8_to_utf16le_async`` (one
    fixed device array per device, shared by every call: calls that overlap
    on one device race)."""
    _dev(data, 1, "data")
    _dev(out, 2, "out")
    cap = out.numel() if out_cap is None else int(out_cap)
    return int(load().convert_utf8_to_utf16le_noalloc_async(_ptr(data), data.numel(), _ptr(out), cap,
                                                         result.data_ptr(), _stream(stream)))


def convert_utf16le_to_utf8_async(data, out, result, out_cap=None, stream=None) -> int:
    _dev(data, 2, "data")
    _dev(out, 1, "out")
    cap = out.numel() if out_cap is None else int(out_cap)
    return int(load().convert_utf16le_to_utf8_async(_ptr(data), data.numel(), _ptr(out), cap,
                                                 result.data_ptr(), _stream(stream)))


# batched conversion: k strings back to back

def results_tensor(k: int, device="cuda") -> torch.Tensor:
    """Device storage for ``k`` ``utf_result`` values (int64[k, 2])."""
    return torch.zeros((max(k, 1), 2), dtype=torch.int64, device=device)


def decode_results(t: torch.Tensor, k: int):
    """``(status int32[k], count int64[k])`` as numpy arrays."""
    v = t[:k].cpu()
    status = (v[:, 0] & 0xFFFFFFFF).to(torch.int64)
    status = torch.where(status >= 1 << 31, status - (1 << 32), status).to(torch.int32)
    return status.numpy(), v[:, 1].numpy()


def convert_utf8_to_utf16le_batch_async(data, offsets, out, out_offsets, results, out_cap=None,
                                        stream=None) -> int:
    """``offsets`` int64[k+1] (device), ``out_offsets`` int64[k+1] (device),
    ``results`` from ``results_tensor(k)``."""
    _dev(data, 1, "data")
    _dev(offsets, 8, "offsets")
    _dev(out_offsets, 8, "out_offsets")
    _dev(out, 2, "out")
    _dev(results, 8, "results")
    k = offsets.numel() - 1
    if k < 0 or out_offsets.numel() < k + 1 or results.numel() < 2 * k:
        raise ValueError("offsets needs k+1 entries, out_offsets k+1, results k")
    cap = out.numel() if out_cap is None else int(out_cap)
    return int(load().convert_utf8_to_utf16le_batch_async(
        _ptr(data), data.numel(), offsets.data_ptr(), k, _ptr(out), cap, out_offsets.data_ptr(),
        results.data_ptr(), _stream(stream)))


def convert_utf16le_to_utf8_batch_async(data, offsets, out, out_offsets, results, out_cap=None,
                                        stream=None) -> int:
    """``data`` 2-byte elements; ``offsets`` int64[k+1] in 16-bit units;
    ``out`` bytes; ``out_offsets`` int64[k+1] (bytes); ``results`` from
    ``results_tensor(k)``."""
    _dev(data, 2, "data")
    _dev(offsets, 8, "offsets")
    _dev(out_offsets, 8, "out_offsets")
    _dev(out, 1, "out")
    _dev(results, 8, "results")
    k = offsets.numel() - 1
    if k < 0 or out_offsets.numel() < k + 1 or results.numel() < 2 * k:
        raise ValueError("offsets needs k+1 entries, out_offsets k+1, results k")
    cap = out.numel() if out_cap is None else int(out_cap)
    return int(load().convert_utf16le_to_utf8_batch_async(
        _ptr(data), data.numel(), offsets.data_ptr(), k, _ptr(out), cap, out_offsets.data_ptr(),
        results.data_ptr(), _stream(stream)))
