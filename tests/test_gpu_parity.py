"""GPU parity: every C-ABI call against the CPU oracle, bit for bit.

Covers every size 0..300, multi-tile buffers with ragged tails, misaligned
input and output pointers, patterns straddling lane / row / wave / tile /
buffer-end boundaries, random invalid byte strings, capacity clamps, the
asynchronous forms, API misuse, and repeatability of the single-pass scan.
"""
import numpy as np
import pytest
import torch

import oracle as O
from tests.gpu_util import guarded_out, to_dev, to_host
from workloads import SCRIPT_MIXES, make_buffer, random_text
from workloads.mixes import UTF8_BAD_PATTERNS

pytestmark = pytest.mark.gpu

MIXES = ("mix1m",) + SCRIPT_MIXES


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2111_08692_amd as G
    G.load()
    return G


# ---------------------------------------------------------------------------
# checkers
# ---------------------------------------------------------------------------

def check_utf8(G, orc, data, in_off=0, out_off=0, cap=None, label=""):
    data = np.ascontiguousarray(data, dtype=np.uint8)
    d = to_dev(data, in_off)
    ov = orc.validate_utf8(data)
    assert G.validate_utf8(d) == ov, ("validate", label)
    need = orc.utf16_length_from_utf8(data)
    assert G.utf16_length_from_utf8(d) == need, ("length", label)
    cap = need if cap is None else cap
    buf, out, sentinel = guarded_out(cap, 2, out_off)
    st, cnt, _ = G.convert_utf8_to_utf16le(d, out=out)
    ost, ocnt, oout = orc.convert_utf8_to_utf16le(data, cap=cap)
    assert (st, cnt) == (ost, ocnt), ("convert", label, (st, cnt), (ost, ocnt))
    got = to_host(out, cap)
    if ost in (O.OK, O.OUTPUT_TOO_SMALL):
        k = min(cap, ocnt)
    else:
        k = min(cap, orc.utf16_length_from_utf8(data[:ocnt]))
    assert np.array_equal(got[:k], oout[:k]), ("output", label, int(np.argmax(got[:k] != oout[:k])))
    whole = to_host(buf, buf.numel())
    assert np.all(whole[:out_off] == sentinel) and np.all(whole[out_off + cap:] == sentinel), ("guard", label)


def check_utf16(G, orc, data, in_off=0, out_off=0, cap=None, label=""):
    data = np.ascontiguousarray(data, dtype=np.uint16)
    d = to_dev(data, in_off)
    ov = orc.validate_utf16le(data)
    assert G.validate_utf16le(d) == ov, ("validate", label)
    need = orc.utf8_length_from_utf16le(data)
    assert G.utf8_length_from_utf16le(d) == need, ("length", label)
    cap = need if cap is None else cap
    buf, out, sentinel = guarded_out(cap, 1, out_off)
    st, cnt, _ = G.convert_utf16le_to_utf8(d, out=out)
    ost, ocnt, oout = orc.convert_utf16le_to_utf8(data, cap=cap)
    assert (st, cnt) == (ost, ocnt), ("convert", label, (st, cnt), (ost, ocnt))
    got = to_host(out, cap)
    if ost in (O.OK, O.OUTPUT_TOO_SMALL):
        k = min(cap, ocnt)
    else:
        k = min(cap, orc.utf8_length_from_utf16le(data[:ocnt]))
    assert np.array_equal(got[:k], oout[:k]), ("output", label, int(np.argmax(got[:k] != oout[:k])))
    whole = to_host(buf, buf.numel())
    assert np.all(whole[:out_off] == sentinel) and np.all(whole[out_off + cap:] == sentinel), ("guard", label)


# ---------------------------------------------------------------------------
# sizes
# ---------------------------------------------------------------------------

def test_every_small_size_utf8(G, orc):
    rng = np.random.default_rng(100)
    for n in range(0, 301):
        mix = MIXES[n % len(MIXES)]
        t = random_text(rng, mix, n + 4)[:n]          # cut anywhere: ragged tails
        check_utf8(G, orc, t, label=f"n={n} {mix}")


def test_every_small_size_utf16(G, orc):
    rng = np.random.default_rng(101)
    for m in range(0, 301):
        mix = MIXES[m % len(MIXES)]
        t = random_text(rng, mix, m + 2, encoding="utf-16-le")[:m]
        check_utf16(G, orc, t, label=f"m={m} {mix}")


@pytest.mark.parametrize("mix", MIXES)
def test_multi_tile_ragged_utf8(G, orc, mix):
    TILE = G.tile_bytes()   # input bytes per workgroup of the kernels
    for size in (TILE - 1, TILE, TILE + 1, 3 * TILE + 7, 100_003, 5 * TILE - 2):
        b = make_buffer(mix, size, seed=size)
        check_utf8(G, orc, b.data, label=f"{mix} {size}")
        bi = make_buffer(mix, size, seed=size, error_rate=2e-5, error_seed=size + 1)
        assert orc.validate_utf8(bi.data)[1] == bi.first_error
        check_utf8(G, orc, bi.data, label=f"{mix} {size} invalid")


@pytest.mark.parametrize("mix", MIXES)
def test_multi_tile_ragged_utf16(G, orc, mix):
    TILE = G.tile_bytes()   # input bytes per workgroup of the kernels
    for size in (TILE - 2, TILE, TILE + 2, 3 * TILE + 6, 100_002, 5 * TILE - 2):
        b = make_buffer(mix, size, seed=size, encoding="utf-16-le")
        check_utf16(G, orc, b.data, label=f"{mix} {size}")
        bi = make_buffer(mix, size, seed=size, encoding="utf-16-le", error_rate=2e-5, error_seed=size + 1)
        assert orc.validate_utf16le(bi.data)[1] == bi.first_error
        check_utf16(G, orc, bi.data, label=f"{mix} {size} invalid")


def test_misaligned_pointers(G, orc):
    b8 = make_buffer("mix1m", 70_001, seed=3).data
    b16 = make_buffer("mix1m", 70_002, seed=4, encoding="utf-16-le").data
    for in_off in range(16):
        for out_off in (0, 1, 3, 5, 7):
            check_utf8(G, orc, b8, in_off=in_off, out_off=out_off, label=f"in+{in_off} out+{out_off}")
    for in_off in range(8):
        for out_off in (0, 1, 2, 7, 13):
            check_utf16(G, orc, b16, in_off=in_off, out_off=out_off, label=f"in+{in_off} out+{out_off}")


# ---------------------------------------------------------------------------
# boundary straddles
# ---------------------------------------------------------------------------

VALID_CHARS = ["A", "é", "߿", "ࠀ", "中", "�", "\U00010000", "\U0001f600", "\U0010ffff"]


def _filler(kind: str, nbytes: int) -> bytes:
    """``nbytes`` of filler text of one script, exact length."""
    unit = {"ascii": "a", "cjk": "中", "emoji": "\U0001f600"}[kind].encode()
    k = nbytes // len(unit)
    return unit * k + b"a" * (nbytes - k * len(unit))


def _utf8_patterns():
    pats = [c.encode() for c in VALID_CHARS]
    rng = np.random.default_rng(7)
    for name, ranges in UTF8_BAD_PATTERNS:
        pats.append(bytes(int(rng.integers(lo, hi + 1)) for lo, hi in ranges))
    pats += [b"\xe4\xb8", b"\xf0\x9f\x98", b"\xc3"]
    return pats


@pytest.mark.parametrize("filler", ["ascii", "cjk", "emoji"])
def test_boundary_straddle_utf8(G, orc, filler):
    TILE = G.tile_bytes()   # input bytes per workgroup of the kernels
    pats = _utf8_patterns()
    for bnd in (16, 1024, 4096, TILE, 2 * TILE):
        for delta in range(-4, 5):
            pos = bnd + delta
            for p in pats:
                data = _filler(filler, pos) + p + _filler(filler, 37)
                check_utf8(G, orc, np.frombuffer(data, dtype=np.uint8), label=f"{bnd}{delta:+d} {p.hex()}")
                # the same pattern at the very end of the buffer
                data = _filler(filler, pos) + p
                check_utf8(G, orc, np.frombuffer(data, dtype=np.uint8), label=f"end {bnd}{delta:+d} {p.hex()}")


@pytest.mark.parametrize("filler", ["ascii", "cjk", "emoji"])
def test_boundary_straddle_utf16(G, orc, filler):
    TILE = G.tile_bytes()   # input bytes per workgroup of the kernels
    pats = [np.frombuffer(c.encode("utf-16-le"), dtype="<u2") for c in VALID_CHARS]
    pats += [np.array(x, dtype=np.uint16) for x in ([0xD800], [0xDBFF], [0xDC00], [0xDFFF], [0xDC00, 0xD800],
                                                    [0xD83D, 0xD83D, 0xDE00])]
    fill = {"ascii": "a", "cjk": "中", "emoji": "\U0001f600"}[filler]
    for bnd in (8, 512, 2048, TILE // 2, TILE):
        for delta in range(-3, 4):
            pos = bnd + delta
            unit = np.frombuffer(fill.encode("utf-16-le"), dtype="<u2")
            k = pos // unit.size
            pre = np.concatenate([np.tile(unit, k), np.full(pos - k * unit.size, 0x61, dtype=np.uint16)])
            post = np.tile(unit, 9)
            for p in pats:
                check_utf16(G, orc, np.concatenate([pre, p, post]).astype(np.uint16), label=f"{bnd}{delta:+d} {p}")
                check_utf16(G, orc, np.concatenate([pre, p]).astype(np.uint16), label=f"end {bnd}{delta:+d} {p}")


def test_ascii_and_surrogate_waves_utf16(G, orc):
    """Waves holding only ASCII words and surrogates take their own encoder:
    pairs straddling dword, lane, row and wave boundaries (ASCII shifts of
    0..9 words), an unpaired high or low word or a reversed pair at those
    places, and one word of another script that makes the wave general."""
    rng = np.random.default_rng(21)
    base = random_text(rng, "emoji", 6000, encoding="utf-16-le")
    assert np.all((base < 0x80) | ((base & 0xF800) == 0xD800))
    for shift in range(10):
        data = np.concatenate([np.full(shift, 0x61, dtype=np.uint16), base]).astype(np.uint16)
        check_utf16(G, orc, data, label=f"shift {shift}")
    smile = [0xD83D, 0xDE00]
    for bnd in (7, 8, 512, 2048, 4096):
        for delta in (-2, -1, 0, 1):
            pos = bnd + delta
            pre = np.full(pos, 0x41, dtype=np.uint16)
            for mid in ([0xD83D], [0xDE00], [0xDE00, 0xD83D], smile, [0x20AC], [0x0101] + smile):
                data = np.concatenate([pre, np.array(mid, dtype=np.uint16), np.tile(smile, 700)]).astype(np.uint16)
                check_utf16(G, orc, data, label=f"{bnd}{delta:+d} {mid}")


# ---------------------------------------------------------------------------
# random invalid inputs
# ---------------------------------------------------------------------------

EDGE8 = np.array([0x00, 0x41, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF, 0xE0, 0xE1,
                  0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8, 0xFF], dtype=np.uint8)


def test_random_edge_bytes(G, orc):
    rng = np.random.default_rng(9)
    for _ in range(1500):
        n = int(rng.integers(1, 40))
        check_utf8(G, orc, EDGE8[rng.integers(0, EDGE8.size, size=n)], label="edge")


def test_random_bytes_long(G, orc):
    TILE = G.tile_bytes()   # input bytes per workgroup of the kernels
    """Uniform random bytes: width up to 2 words per byte (stage clamp)."""
    rng = np.random.default_rng(10)
    for n in (5000, TILE, 3 * TILE + 5):
        check_utf8(G, orc, rng.integers(0, 256, size=n, dtype=np.uint8), label=f"random {n}")
        check_utf8(G, orc, rng.integers(0xF0, 0x100, size=n, dtype=np.uint8), label=f"high {n}")
        w = rng.integers(0xD700, 0xE100, size=n // 2).astype(np.uint16)
        check_utf16(G, orc, w, label=f"surrogates {n}")


def test_mutated_text(G, orc):
    rng = np.random.default_rng(12)
    for it in range(300):
        t = bytearray(random_text(rng, MIXES[it % len(MIXES)], int(rng.integers(1, 3000))).tobytes())
        for _ in range(int(rng.integers(1, 4))):
            p = int(rng.integers(0, len(t)))
            t[p] = int(EDGE8[rng.integers(0, EDGE8.size)])
        check_utf8(G, orc, np.frombuffer(bytes(t), dtype=np.uint8), label=f"mutated {it}")


# ---------------------------------------------------------------------------
# capacity, async, misuse, repeatability
# ---------------------------------------------------------------------------

def test_capacity_clamp(G, orc):
    rng = np.random.default_rng(13)
    t8 = random_text(rng, "mix1m", 30000)
    need = orc.utf16_length_from_utf8(t8)
    for cap in (0, 1, 2, 7, 8, 9, need // 3, need - 1, need):
        check_utf8(G, orc, t8, cap=cap, label=f"cap {cap}")
    t16 = random_text(rng, "emoji", 30000, encoding="utf-16-le")
    need = orc.utf8_length_from_utf16le(t16)
    for cap in (0, 1, 2, 3, 15, 16, 17, need // 2, need - 1, need):
        check_utf16(G, orc, t16, cap=cap, label=f"cap {cap}")


def test_async_forms(G, orc):
    rng = np.random.default_rng(14)
    t8 = random_text(rng, "mix1m", 50000)
    bad = t8.copy()
    bad[33333] = 0xFF
    for data in (t8, bad, t8[:0]):
        d = to_dev(data)
        r = G.result_tensor()
        assert G.validate_utf8_async(d, r) == 0
        assert G.decode_result(r) == orc.validate_utf8(data)
        lr = torch.zeros(1, dtype=torch.int64, device="cuda")
        assert G.utf16_length_from_utf8_async(d, lr) == 0
        assert int(lr.item()) == orc.utf16_length_from_utf8(data)
        out = torch.empty(max(data.size, 1), dtype=torch.int16, device="cuda")
        assert G.convert_utf8_to_utf16le_async(d, out, r) == 0
        st, cnt, oo = orc.convert_utf8_to_utf16le(data)
        assert G.decode_result(r) == (st, cnt)
        if st == 0:
            assert np.array_equal(to_host(out, cnt), oo[:cnt])
    t16 = random_text(rng, "emoji", 40000, encoding="utf-16-le")
    d = to_dev(t16)
    r = G.result_tensor()
    assert G.validate_utf16le_async(d, r) == 0
    assert G.decode_result(r) == orc.validate_utf16le(t16)
    lr = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert G.utf8_length_from_utf16le_async(d, lr) == 0
    assert int(lr.item()) == orc.utf8_length_from_utf16le(t16)
    out = torch.empty(3 * t16.size, dtype=torch.uint8, device="cuda")
    assert G.convert_utf16le_to_utf8_async(d, out, r) == 0
    st, cnt, oo = orc.convert_utf16le_to_utf8(t16)
    assert G.decode_result(r) == (st, cnt) and np.array_equal(to_host(out, cnt), oo[:cnt])


def test_api_misuse(G):
    L = G.load()
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    p = buf.data_ptr()
    s = torch.cuda.current_stream().cuda_stream
    assert L.validate_utf16le(p + 1, 4, s).status == G.ERR_ALIGN
    assert L.convert_utf8_to_utf16le(p, 4, p + 1, 4, s).status == G.ERR_ALIGN
    assert L.validate_utf8(None, 4, s).status == G.ERR_NULL
    assert L.validate_utf8(None, 0, s).status == G.OK
    assert L.convert_utf8_to_utf16le(p, 4, None, 4, s).status == G.ERR_NULL
    assert L.validate_utf8(p, 1 << 40, s).status == G.ERR_TOO_BIG
    assert L.utf16_length_from_utf8(None, 5, s) == (1 << 64) - 1


def test_repeatable_many_tiles(G, orc):
    """The look-back scan gives identical output on every run."""
    b = make_buffer("emoji", 6 << 20, seed=77).data
    d = to_dev(b)
    st0, c0, out0 = G.convert_utf8_to_utf16le(d)
    ost, oc, oo = orc.convert_utf8_to_utf16le(b)
    assert (st0, c0) == (ost, oc)
    ref = to_host(out0, c0)
    assert np.array_equal(ref, oo[:oc])
    for _ in range(20):
        st, c, out = G.convert_utf8_to_utf16le(d)
        assert (st, c) == (st0, c0) and torch.equal(out[:c], out0[:c])
