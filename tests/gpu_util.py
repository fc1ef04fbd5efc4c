"""Helpers shared by the GPU parity tests (no codec logic here).

UTF-16 data lives on the device as ``torch.int16`` (2-byte elements; the
library only looks at the bytes) and on the host as numpy ``uint16``.
"""
import numpy as np
import torch


def to_dev(a: np.ndarray, offset_units: int = 0, slack: int = 64) -> torch.Tensor:
    """Copy ``a`` to the GPU, starting ``offset_units`` elements into a fresh
    allocation (to test misaligned pointers); returns the view."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint8:
        dt, host = torch.uint8, a
    elif a.dtype == np.uint16:
        dt, host = torch.int16, a.view(np.int16)
    else:
        raise TypeError(a.dtype)
    buf = torch.zeros(a.size + offset_units + slack, dtype=dt, device="cuda")
    view = buf[offset_units:offset_units + a.size]
    if a.size:
        view.copy_(torch.from_numpy(np.array(host, copy=True)).to("cuda"))
    return view


def to_host(t: torch.Tensor, n: int) -> np.ndarray:
    a = t[:n].cpu().numpy()
    return a.view(np.uint16) if a.dtype == np.int16 else a


def guarded_out(n: int, elem: int, offset_units: int = 0, guard: int = 64):
    """Output buffer of ``n`` elements with sentinel elements after it (and
    ``offset_units`` before it) to detect writes outside the capacity.
    Returns ``(whole buffer, view, sentinel value)``."""
    if elem == 1:
        buf = torch.full((offset_units + n + guard,), 0xA5, dtype=torch.uint8, device="cuda")
        sentinel = 0xA5
    else:
        buf = torch.full((offset_units + n + guard,), -0x5A5B, dtype=torch.int16, device="cuda")
        sentinel = 0xA5A5
    return buf, buf[offset_units:offset_units + n], sentinel


def out16(n: int) -> torch.Tensor:
    return torch.empty(max(n, 1), dtype=torch.int16, device="cuda")


def out8(n: int) -> torch.Tensor:
    return torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
