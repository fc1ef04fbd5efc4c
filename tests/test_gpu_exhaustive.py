"""Every 4-byte UTF-8 string and every 2-unit UTF-16LE string through the
device, against the closed forms of the paper's Section 3 rules and the
oracle.

The 2^32 strings of each enumeration go through the batched conversion,
2^28 strings (1 GiB of input) per call: string i is the four bytes of i,
most significant first (UTF-8), or the units (i >> 16, i & 0xFFFF)
(UTF-16LE).  For every call, each string's status and count (output units,
or the first-error offset) must equal the oracle's, and the output units of
the valid strings must give the same weighted sums (tests/exhaustive_parts.py).
Over all calls the number of valid strings must be V(4) = 383 270 912 for
UTF-8 and W(2) = 4 031 774 720 for UTF-16LE, and the histogram of
first-error offsets the closed form of the valid-prefix counts.
"""
import multiprocessing as mp
import sys
from collections import Counter
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import torch

from tests.exhaustive_parts import SLOTS, part
from tests.test_oracle_pins import N8, N16, error_histogram

pytestmark = pytest.mark.gpu

CALL = 1 << 28          # strings per batched call
PART = 1 << 23          # strings per oracle part (and per device digest)
GROUPS = 4              # test cases per enumeration, 4 calls each
CALLS = (1 << 32) // CALL


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available()
    import paper_2111_08692_amd as G
    G.load()
    return G


@pytest.fixture(scope="module")
def pool():
    ex = ProcessPoolExecutor(max_workers=16, mp_context=mp.get_context("spawn"))
    yield ex
    ex.shutdown()


TALLY = {"utf-8": {"calls": set(), "valid": 0, "hist": Counter()},
         "utf-16-le": {"calls": set(), "valid": 0, "hist": Counter()}}


class Device:
    """Buffers of one enumeration, reused by every call."""

    def __init__(self, G, encoding):
        self.G, self.enc = G, encoding
        self.width = 4 if encoding == "utf-8" else 2
        unit = 1 if encoding == "utf-8" else 2
        self.data = torch.empty(CALL * self.width * unit, dtype=torch.uint8, device="cuda")
        self.offsets = torch.arange(0, self.width * CALL + 1, self.width, dtype=torch.int64, device="cuda")
        self.oo = torch.empty(CALL + 1, dtype=torch.int64, device="cuda")
        self.res = G.results_tensor(CALL)
        # every byte >= F0 counts two words; at most 3 bytes per UTF-16 unit
        self.cap = 2 * self.width * CALL if encoding == "utf-8" else 3 * self.width * CALL
        self.out = torch.empty(self.cap, dtype=torch.int16 if encoding == "utf-8" else torch.uint8, device="cuda")

    def fill(self, lo):
        i = torch.arange(lo, lo + CALL, dtype=torch.int64, device="cuda")
        b = self.data.view(CALL, 4)
        if self.enc == "utf-8":   # bytes of i, most significant first
            for j in range(4):
                b[:, j] = ((i >> (24 - 8 * j)) & 0xFF).to(torch.uint8)
        else:                     # units i >> 16, i & 0xFFFF, little-endian
            for j, sh in enumerate((16, 24, 0, 8)):
                b[:, j] = ((i >> sh) & 0xFF).to(torch.uint8)
        del i

    def run(self, lo):
        self.fill(lo)
        d = self.data if self.enc == "utf-8" else self.data.view(torch.int16)
        conv = (self.G.convert_utf8_to_utf16le_batch_async if self.enc == "utf-8"
                else self.G.convert_utf16le_to_utf8_batch_async)
        assert conv(d, self.offsets, self.out, self.oo, self.res) == 0
        torch.cuda.synchronize()
        st = (self.res[:, 0] & 0xFFFFFFFF)
        cnt = self.res[:, 1]
        assert int(st.max()) <= 8 and int(cnt.max()) <= 7   # no OUTPUT_TOO_SMALL, no misuse status
        codes = (st * 8 + cnt).to(torch.uint8).cpu().numpy()
        digests = {}
        for p0 in range(0, CALL, PART):
            sl = slice(p0, p0 + PART)
            valid = st[sl] == 0
            idx = torch.nonzero(valid).squeeze(1)
            w = ((idx + lo + p0) & 0xFFFFF) + 1
            c = cnt[sl][idx]
            base = self.oo[sl][idx]
            dg = []
            for j in range(SLOTS[self.enc]):
                has = c > j
                u = torch.zeros_like(idx)
                pos = torch.where(has, base + j, torch.zeros_like(base))
                g = self.out[pos].to(torch.int64) & (0xFFFF if self.enc == "utf-8" else 0xFF)
                u = torch.where(has, g, u)
                dg += [int((u * w).sum()), int(u.sum())]
            digests[lo + p0] = dg
        return codes, digests


_dev = {}


def _device(G, enc):
    if enc not in _dev:
        _dev.clear()
        torch.cuda.empty_cache()
        _dev[enc] = Device(G, enc)
    return _dev[enc]


def _check_calls(G, pool, enc, group):
    dev = _device(G, enc)
    tally = TALLY[enc]
    for c in range(group * CALLS // GROUPS, (group + 1) * CALLS // GROUPS):
        lo = c * CALL
        futs = [pool.submit(part, enc, lo + p0, lo + p0 + PART) for p0 in range(0, CALL, PART)]
        print(f"[exhaustive] {enc} call {c} strings {lo:#x}..{lo + CALL:#x}", file=sys.stderr, flush=True)
        codes, digests = dev.run(lo)
        for f in futs:
            plo, pcodes, pdig = f.result()
            got = codes[plo - lo:plo - lo + PART]
            if not np.array_equal(got, pcodes):
                bad = int(np.nonzero(got != pcodes)[0][0])
                raise AssertionError(f"{enc} string {plo + bad:#x}: device code {got[bad]} oracle {pcodes[bad]}")
            assert digests[plo] == pdig, (enc, hex(plo))
        st = codes >> 3
        tally["valid"] += int((st == 0).sum())
        tally["hist"].update(dict(enumerate(np.bincount((codes[st != 0] & 7).astype(np.int64)).tolist())))
        tally["calls"].add(c)


@pytest.mark.parametrize("group", range(GROUPS))
def test_all_4byte_utf8_strings(G, pool, group):
    _check_calls(G, pool, "utf-8", group)


def test_all_4byte_utf8_closed_forms():
    t = TALLY["utf-8"]
    assert t["calls"] == set(range(CALLS)), "run with every group of the enumeration"
    v, hist = error_histogram(4, N8, 256)
    assert t["valid"] == v == 383_270_912
    assert {p: t["hist"].get(p, 0) for p in range(4)} == hist and set(t["hist"]) <= set(range(4))


@pytest.mark.parametrize("group", range(GROUPS))
def test_all_2unit_utf16_strings(G, pool, group):
    _check_calls(G, pool, "utf-16-le", group)


def test_all_2unit_utf16_closed_forms():
    t = TALLY["utf-16-le"]
    assert t["calls"] == set(range(CALLS)), "run with every group of the enumeration"
    v, hist = error_histogram(2, N16, 65536)
    assert t["valid"] == v == 4_031_774_720
    assert {p: t["hist"].get(p, 0) for p in range(2)} == hist and set(t["hist"]) <= set(range(2))
