"""Oracle side of the exhaustive device tests (test infrastructure, CPU
only, no torch): every 4-byte UTF-8 string and every 2-unit UTF-16LE
string, enumerated part by part in worker processes.

String i of the UTF-8 enumeration is the four bytes of i, most significant
first; string i of the UTF-16LE enumeration is the two units (i >> 16,
i & 0xFFFF).  For a part [lo, hi) of indices a worker converts every string
on its own with the oracle's batched call and returns

* ``codes``: one byte per string, status * 8 + count (count = output
  units of a valid string, first-error offset of an invalid one);
* ``digest``: for output unit slot j of a string (j < ``SLOTS``), the sum
  over the part's valid strings of unit j times (i mod 2^20) + 1, and the
  plain sum of unit j: exact integers, computed the same way on the device.
"""
import numpy as np

import oracle as O

SLOTS = {"utf-8": 4, "utf-16-le": 6}   # most output units of one string


def strings(encoding: str, lo: int, hi: int) -> np.ndarray:
    """The strings lo .. hi-1 back to back (uint8 for UTF-8, uint16 units)."""
    i = np.arange(lo, hi, dtype=np.uint64)
    if encoding == "utf-8":
        return i.astype(">u4").view(np.uint8)
    u = np.empty((hi - lo, 2), dtype=np.uint16)
    u[:, 0] = (i >> np.uint64(16)).astype(np.uint16)
    u[:, 1] = (i & np.uint64(0xFFFF)).astype(np.uint16)
    return u.reshape(-1)


def digest(units: np.ndarray, out_offsets: np.ndarray, count: np.ndarray, valid: np.ndarray, lo: int,
           slots: int) -> list:
    """Weighted and plain sums of each output slot over the valid strings."""
    idx = np.nonzero(valid)[0]
    w = ((idx.astype(np.int64) + lo) & 0xFFFFF) + 1
    res = []
    for j in range(slots):
        has = count[idx] > j
        u = np.zeros(idx.size, dtype=np.int64)
        u[has] = units[out_offsets[idx[has]] + j]
        res += [int((u * w).sum()), int(u.sum())]
    return res


def part(encoding: str, lo: int, hi: int):
    """(lo, codes, digest) of strings lo .. hi-1."""
    data = strings(encoding, lo, hi)
    width = 4 if encoding == "utf-8" else 2
    offsets = np.arange(0, width * (hi - lo) + 1, width, dtype=np.int64)
    conv = O.convert_utf8_to_utf16le_batch if encoding == "utf-8" else O.convert_utf16le_to_utf8_batch
    st, cnt, out, oo = conv(data, offsets)
    codes = (st.astype(np.int64) * 8 + cnt.astype(np.int64)).astype(np.uint8)
    valid = st == O.OK
    return lo, codes, digest(out.astype(np.int64), oo, cnt.astype(np.int64), valid, lo, SLOTS[encoding])
