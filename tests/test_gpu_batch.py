"""GPU parity of the batched UTF-8 -> UTF-16LE call against the CPU oracle.

Every string of a batch is its own input (its first byte continues nothing
before it, its last character must end inside it), so the cases put
characters, errors and empty strings across string, lane, row, wave and tile
boundaries, and check statuses, first-error positions, compact output
offsets and the words of every valid string, bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle as O
from tests.gpu_util import guarded_out, to_dev, to_host
from workloads import random_text
from workloads.mixes import SEED_BATCH, make_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2111_08692_amd as G
    G.load()
    return G


def run_batch(G, data, offsets, in_off=0, cap=None, out_off=0):
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = offsets.size - 1
    d = to_dev(data, in_off)
    offs = torch.from_numpy(offsets).to("cuda")
    cap = int(cap)
    buf, out, sentinel = guarded_out(cap, 2, out_off)
    oo = torch.full((k + 1,), -7, dtype=torch.int64, device="cuda")
    res = G.results_tensor(k)
    rc = G.convert_utf8_to_utf16le_batch_async(d, offs, out, oo, res, out_cap=cap)
    torch.cuda.synchronize()
    st, cnt = G.decode_results(res, k)
    return rc, st, cnt, oo.cpu().numpy(), to_host(out, cap), to_host(buf, buf.numel()), sentinel


def check_batch(G, orc, data, offsets, in_off=0, cap=None, out_off=0, label=""):
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = offsets.size - 1
    ost, ocnt, oout, ooff = orc.convert_utf8_to_utf16le_batch(data, offsets)
    total = int(ooff[-1])
    cap = total if cap is None else int(cap)
    rc, st, cnt, goff, got, whole, sentinel = run_batch(G, data, offsets, in_off, cap, out_off)
    assert rc == 0, (label, rc)
    assert np.array_equal(goff, ooff), (label, "out_offsets", int(np.argmax(goff != ooff)))
    # a valid string whose words do not all fit below the capacity
    est = np.where((ost == O.OK) & (ooff[1:] > cap), O.OUTPUT_TOO_SMALL, ost)
    bad = np.nonzero((st != est) | (cnt != ocnt))[0]
    assert bad.size == 0, (label, "results", int(bad[0]), (int(st[bad[0]]), int(cnt[bad[0]])),
                           (int(est[bad[0]]), int(ocnt[bad[0]])))
    # words of valid strings (below the capacity) are exact
    lens = np.diff(ooff)
    valid_word = np.repeat(ost == O.OK, lens)[:cap]
    diff = np.nonzero(valid_word & (got[:min(cap, total)] != oout[:cap]))[0] if total else np.zeros(0)
    assert diff.size == 0, (label, "output word", int(diff[0]))
    assert np.all(whole[:out_off] == sentinel) and np.all(whole[out_off + cap:] == sentinel), (label, "guard")
    return st


def pack(strings):
    parts = [np.frombuffer(bytes(s), dtype=np.uint8) for s in strings]
    offsets = np.zeros(len(parts) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([p.size for p in parts])
    data = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint8)
    return data, offsets


def test_small_hand_cases(G, orc):
    euro = "€".encode()            # E2 82 AC
    smile = "😀".encode()          # F0 9F 98 80
    strings = [
        b"", b"a", b"", b"", "é".encode(), euro, smile,
        euro[:1], euro[1:],        # a character split across two strings: both invalid
        smile[:3], smile[3:],      # same, four-byte character
        b"abc" + euro[:2], euro[2:] + b"xyz",
        b"\x80", b"\xc3", b"\xff", b"\xed\xa0\x80", b"\xc0\xaf", b"\xf4\x90\x80\x80",
        b"plain ascii " * 5, b"",
    ]
    data, offsets = pack(strings)
    st = check_batch(G, orc, data, offsets, label="hand")
    assert st[7] == O.TOO_SHORT and st[8] == O.TOO_LONG and st[9] == O.TOO_SHORT and st[10] == O.TOO_LONG


def test_empty_batches(G, orc):
    # k == 0
    data = np.zeros(0, dtype=np.uint8)
    offs = torch.zeros(1, dtype=torch.int64, device="cuda")
    oo = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    res = G.results_tensor(0)
    out = torch.zeros(1, dtype=torch.int16, device="cuda")
    assert G.convert_utf8_to_utf16le_batch_async(to_dev(data), offs, out, oo, res) == 0
    torch.cuda.synchronize()
    assert int(oo[0]) == 0
    # k == 0 cannot partition a non-empty input
    d1 = to_dev(np.frombuffer(b"abc", dtype=np.uint8))
    assert G.convert_utf8_to_utf16le_batch_async(d1, offs, out, oo, res) == G.ERR_OFFSETS
    # k > 0 strings, all empty (n == 0)
    check_batch(G, orc, data, np.zeros(17, dtype=np.int64), label="all empty")
    # one long string == the single-buffer call
    rng = np.random.default_rng(5)
    t = random_text(rng, "mix1m", 50_000)
    check_batch(G, orc, t, np.array([0, t.size]), label="one string")


@pytest.mark.parametrize("mix", ["ascii", "latin", "cyrillic", "cjk", "emoji", "mix1m"])
@pytest.mark.parametrize("median", [3, 40, 700])
def test_generated_batches(G, orc, mix, median):
    b = make_batch(k=600, seed=SEED_BATCH + 11 + median, median=median, sigma=1.2, lo=0, hi=40_000,
                   error_fraction=0.2, mixes=(mix,))
    check_batch(G, orc, b.data, b.offsets, label=f"{mix}/{median}")


def test_mixed_with_misalignment_and_capacity(G, orc):
    b = make_batch(k=3000, seed=SEED_BATCH + 3, median=120, sigma=1.5, lo=0, hi=100_000,
                   error_fraction=0.05)
    for in_off in (0, 1, 7, 13):
        check_batch(G, orc, b.data, b.offsets, in_off=in_off, out_off=in_off % 3, label=f"off{in_off}")
    total = int(orc.convert_utf8_to_utf16le_batch(b.data, b.offsets)[3][-1])
    for cap in (0, 1, total // 3, total - 1):
        check_batch(G, orc, b.data, b.offsets, cap=cap, label=f"cap{cap}")


def test_random_bytes_and_boundaries(G, orc):
    rng = np.random.default_rng(77)
    strings = []
    for i in range(4000):
        kind = i % 5
        n = int(rng.integers(0, 40))
        if kind == 0:
            strings.append(rng.integers(0, 256, size=n, dtype=np.uint8).tobytes())
        elif kind == 1:   # bytes drawn from the interesting values
            vals = np.array([0x41, 0x80, 0xBF, 0xC2, 0xDF, 0xE0, 0xED, 0xEF, 0xF0, 0xF4, 0xF5, 0xC0], np.uint8)
            strings.append(rng.choice(vals, size=n).tobytes())
        else:
            t = random_text(rng, "mix1m", n)
            strings.append(t.tobytes())
    data, offsets = pack(strings)
    st = check_batch(G, orc, data, offsets, label="random")
    assert (st == O.OK).sum() > 1000 and (st != O.OK).sum() > 500


def test_stage_overflow_then_valid(G, orc):
    # long runs of F5 (two words each, no continuation bytes) announce more
    # words than a wave stages; the valid strings after them in the same
    # wave, row and lane must still be exact
    rng = np.random.default_rng(3)
    strings = []
    for i in range(200):
        strings.append(b"\xf5" * int(rng.integers(200, 3000)))
        strings.append(random_text(rng, "emoji", int(rng.integers(1, 60))).tobytes())
        strings.append(b"\xf0" * int(rng.integers(1, 20)))
        strings.append(random_text(rng, "mix1m", int(rng.integers(1, 60))).tobytes())
    data, offsets = pack(strings)
    st = check_batch(G, orc, data, offsets, label="overflow")
    assert np.all(st[0::4] == O.TOO_SHORT) and np.all(st[1::4] == O.OK)


def test_strings_at_every_alignment_of_a_chunk(G, orc):
    # a valid string starting at each position of a 16-byte chunk, after an
    # invalid string whose last lead announces bytes past its end
    rng = np.random.default_rng(9)
    strings = []
    for pad in range(64):
        strings.append(b"x" * pad + b"\xe2\x82")
        strings.append(random_text(rng, "cjk", 9).tobytes())
        strings.append(b"\x82" * (pad % 5) + b"ok")
        strings.append("ñ".encode() * (pad % 7))
    data, offsets = pack(strings)
    check_batch(G, orc, data, offsets, label="alignment")


def test_bad_offsets_then_good_call(G, orc):
    b = make_batch(k=500, seed=SEED_BATCH + 5, median=100, sigma=1.0, lo=0, hi=5000, error_fraction=0.1)
    k = b.offsets.size - 1
    dec = b.offsets.copy()
    dec[11] = dec[10] - 1                    # string 10 ends before it starts
    neg = b.offsets.copy()
    neg[3] = -1
    for bad in (np.r_[1, b.offsets[1:]], np.r_[b.offsets[:-1], b.data.size - 1], dec, neg):
        rc, st, cnt, goff, *_ = run_batch(G, b.data, bad, cap=b.data.size)
        assert rc == 0
        assert np.all(st == G.ERR_OFFSETS) and np.all(cnt == 0) and np.all(goff == 0)
    # the library's per-call state is clean again
    check_batch(G, orc, b.data, b.offsets, label="after bad offsets")
    check_batch(G, orc, b.data, b.offsets, label="again")
    assert k == 500


def test_scrambled_offsets_over_invalid_bytes(G, orc):
    """Offsets that are not a partition, over bytes full of errors: flagged
    waves look up the owners of their errors in span owners that the bad
    offsets leave unset (or set by an earlier call with many more strings);
    every string reports ERR_OFFSETS and the library is clean afterwards."""
    rng = np.random.default_rng(91)
    data = rng.integers(0, 256, size=3 << 20, dtype=np.uint8)
    n = data.size
    many = np.r_[0, np.sort(rng.integers(0, n, size=19_999)), n].astype(np.int64)   # valid, 20 000 strings
    check_batch(G, orc, data, many, label="many strings first")
    for k in (50, 3000):
        bad = rng.integers(0, n, size=k + 1).astype(np.int64)   # unsorted
        bad[0], bad[-1] = 0, n
        rc, st, cnt, goff, *_ = run_batch(G, data, bad, cap=n)
        assert rc == 0 and np.all(st == G.ERR_OFFSETS) and np.all(cnt == 0) and np.all(goff == 0), k
        d16 = rng.integers(0xD000, 0xE000, size=n // 2).astype(np.uint16)
        bad16 = rng.integers(0, n // 2, size=k + 1).astype(np.int64)
        bad16[0], bad16[-1] = 0, n // 2
        rc, st, cnt, goff, *_ = run_batch16(G, d16, bad16, cap=3 * d16.size)
        assert rc == 0 and np.all(st == G.ERR_OFFSETS) and np.all(goff == 0), k
    check_batch(G, orc, data, many, label="many strings after")


def test_full_size_batch(G, orc):
    """100 000 strings, log-normal lengths (median 256 bytes, sigma 1.5,
    16 B .. 1 MiB), one script mix each, 1% with one injected error."""
    b = make_batch()
    check_batch(G, orc, b.data, b.offsets, label="full")


# ---------------------------------------------------------------------------
# UTF-16LE -> UTF-8
# ---------------------------------------------------------------------------

def run_batch16(G, data, offsets, in_off=0, cap=None, out_off=0):
    data = np.ascontiguousarray(data, dtype=np.uint16)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = offsets.size - 1
    d = to_dev(data, in_off)
    offs = torch.from_numpy(offsets).to("cuda")
    cap = int(cap)
    buf, out, sentinel = guarded_out(cap, 1, out_off)
    oo = torch.full((k + 1,), -7, dtype=torch.int64, device="cuda")
    res = G.results_tensor(k)
    rc = G.convert_utf16le_to_utf8_batch_async(d, offs, out, oo, res, out_cap=cap)
    torch.cuda.synchronize()
    st, cnt = G.decode_results(res, k)
    return rc, st, cnt, oo.cpu().numpy(), to_host(out, cap), to_host(buf, buf.numel()), sentinel


def check_batch16(G, orc, data, offsets, in_off=0, cap=None, out_off=0, label=""):
    data = np.ascontiguousarray(data, dtype=np.uint16)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    ost, ocnt, oout, ooff = orc.convert_utf16le_to_utf8_batch(data, offsets)
    total = int(ooff[-1])
    cap = total if cap is None else int(cap)
    rc, st, cnt, goff, got, whole, sentinel = run_batch16(G, data, offsets, in_off, cap, out_off)
    assert rc == 0, (label, rc)
    assert np.array_equal(goff, ooff), (label, "out_offsets", int(np.argmax(goff != ooff)))
    est = np.where((ost == O.OK) & (ooff[1:] > cap), O.OUTPUT_TOO_SMALL, ost)
    bad = np.nonzero((st != est) | (cnt != ocnt))[0]
    assert bad.size == 0, (label, "results", int(bad[0]), (int(st[bad[0]]), int(cnt[bad[0]])),
                           (int(est[bad[0]]), int(ocnt[bad[0]])))
    lens = np.diff(ooff)
    valid_byte = np.repeat(ost == O.OK, lens)[:cap]
    diff = np.nonzero(valid_byte & (got[:min(cap, total)] != oout[:cap]))[0] if total else np.zeros(0)
    assert diff.size == 0, (label, "output byte", int(diff[0]))
    assert np.all(whole[:out_off] == sentinel) and np.all(whole[out_off + cap:] == sentinel), (label, "guard")
    return st


def pack16(strings):
    parts = [np.asarray(s, dtype=np.uint16) for s in strings]
    offsets = np.zeros(len(parts) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([p.size for p in parts])
    data = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint16)
    return data, offsets


def u16(text):
    return list(np.frombuffer(text.encode("utf-16-le"), dtype="<u2"))


def test_small_hand_cases16(G, orc):
    smile = u16("😀")   # D83D DE00
    strings = [[], u16("a"), [], u16("é€"), smile, smile[:1], smile[1:], u16("ab") + smile[:1],
               smile[1:] + u16("cd"), [0xDC00], [0xD800], [0xD800, 0x41], [0x41, 0xDFFF], u16("plain " * 7), []]
    data, offsets = pack16(strings)
    st = check_batch16(G, orc, data, offsets, label="hand16")
    assert st[5] == O.UNPAIRED_HIGH and st[6] == O.UNPAIRED_LOW and st[7] == O.UNPAIRED_HIGH
    assert st[8] == O.UNPAIRED_LOW


@pytest.mark.parametrize("mix", ["ascii", "latin", "cyrillic", "cjk", "emoji", "mix1m"])
@pytest.mark.parametrize("median", [4, 60, 900])
def test_generated_batches16(G, orc, mix, median):
    b = make_batch(k=600, seed=SEED_BATCH + 31 + median, encoding="utf-16-le", median=median, sigma=1.2, lo=0,
                   hi=40_000, error_fraction=0.2, mixes=(mix,))
    check_batch16(G, orc, b.data, b.offsets, label=f"16/{mix}/{median}")


def test_random_units_and_alignment16(G, orc):
    rng = np.random.default_rng(78)
    strings = []
    vals = np.array([0x41, 0x7F, 0x80, 0x7FF, 0x800, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xE000, 0xFFFF],
                    np.uint16)
    for i in range(4000):
        n = int(rng.integers(0, 30))
        if i % 3 == 0:
            strings.append(rng.choice(vals, size=n))
        else:
            strings.append(random_text(rng, "emoji" if i % 2 else "mix1m", n, encoding="utf-16-le"))
    data, offsets = pack16(strings)
    for in_off in (0, 1, 5):
        st = check_batch16(G, orc, data, offsets, in_off=in_off, out_off=in_off, label=f"rand16/{in_off}")
    assert (st == O.OK).sum() > 1500 and (st != O.OK).sum() > 300
    total = int(orc.convert_utf16le_to_utf8_batch(data, offsets)[3][-1])
    for cap in (0, total // 2, total - 1):
        check_batch16(G, orc, data, offsets, cap=cap, label=f"cap16/{cap}")


def test_bad_offsets_then_good_call16(G, orc):
    b = make_batch(k=400, seed=SEED_BATCH + 41, encoding="utf-16-le", median=100, sigma=1.0, lo=0, hi=5000,
                   error_fraction=0.1)
    dec = b.offsets.copy()
    dec[11] = dec[10] - 1
    rc, st, cnt, goff, *_ = run_batch16(G, b.data, dec, cap=3 * b.data.size)
    assert rc == 0 and np.all(st == G.ERR_OFFSETS) and np.all(goff == 0)
    check_batch16(G, orc, b.data, b.offsets, label="16 after bad offsets")
    check_batch16(G, orc, b.data, b.offsets, label="16 again")


def test_full_size_batch16(G, orc):
    """100 000 UTF-16LE strings, the same length distribution as the UTF-8 batch."""
    b = make_batch(encoding="utf-16-le")
    check_batch16(G, orc, b.data, b.offsets, label="full16")
