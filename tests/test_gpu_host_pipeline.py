"""Pipelined host-memory conversions against the oracle: chunk cuts at every
kind of boundary, errors just before, at and after cuts, bit-exact (on an
error, the output of the valid prefix)."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import make_buffer, random_text

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2111_08692_amd.host_pipeline import HostPipeline
    return {c: HostPipeline(chunk_bytes=c, nstreams=3) for c in (4096, 1 << 16, 1 << 20)}


def check8(p, orc, data):
    st, cnt, out = p.convert_utf8_to_utf16le(data)
    ost, ocnt, oout = orc.convert_utf8_to_utf16le(data)
    assert (st, cnt) == (ost, ocnt)
    n = ocnt if ost == O.OK else orc.utf16_length_from_utf8(data[:ocnt])   # words of the valid prefix
    assert out.size == n and np.array_equal(out, oout[:n])


def check16(p, orc, data):
    st, cnt, out = p.convert_utf16le_to_utf8(data)
    ost, ocnt, oout = orc.convert_utf16le_to_utf8(data)
    assert (st, cnt) == (ost, ocnt)
    n = ocnt if ost == O.OK else orc.utf8_length_from_utf16le(data[:ocnt])   # bytes of the valid prefix
    assert out.size == n and np.array_equal(out, oout[:n])


@pytest.mark.parametrize("mix", ["mix1m", "cjk", "emoji", "ascii"])
def test_valid(P, orc, mix):
    b8 = make_buffer(mix, 3 << 20, 77).data
    b16 = make_buffer(mix, 3 << 20, 78, encoding="utf-16-le").data
    for p in P.values():
        check8(p, orc, b8)
        check16(p, orc, b16)
    check8(P[4096], orc, b8[:0])
    check16(P[4096], orc, b16[:0])


def test_errors_around_cuts(P, orc):
    rng = np.random.default_rng(3)
    base8 = random_text(rng, "mix1m", 60000)
    base16 = random_text(rng, "emoji", 60000, encoding="utf-16-le")
    p = P[4096]
    for pos in (4093, 4094, 4095, 4096, 4097, 4098, 8191, 12290, base8.size - 1):
        for bad in (0xFF, 0x80, 0xC3, 0xF0):
            t = base8.copy()
            t[pos] = bad
            check8(p, orc, t)
    # a long run of continuation bytes across a cut
    t = base8.copy()
    t[4090:4110] = 0x80
    check8(p, orc, t)
    for pos in (2045, 2046, 2047, 2048, 2049, 4096, base16.size - 1):
        for bad in (0xD800, 0xDC00, 0xDBFF):
            t = base16.copy()
            t[pos] = bad
            check16(p, orc, t)
