"""Pins of the CPU oracle against facts that do not come from the oracle.

* closed-form counts of valid buffers and of first-error positions, from
  the code-point ranges of the paper's Section 3;
* exhaustive enumeration of every scalar value and of every 1-, 2- and
  3-byte buffer;
* CPython's strict ``utf-8`` / ``utf-16-le`` codecs (independent code,
  called, not copied) on seeded random and mutated inputs;
* hand-derived fixtures under ``tests/golden/`` (each line cites the rule);
* invariants: round trip, concatenation, prefix property, length query ==
  units written.
"""
import os
import struct

import numpy as np
import pytest

import oracle as O
from workloads import SCRIPT_MIXES, random_text

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NAMES = {v: k for k, v in O.STATUS_NAMES.items()}

# Number of valid characters of each length (Section 3 value ranges):
#   UTF-8: U+0..7F, U+80..7FF, U+800..FFFF minus 2048 surrogates, U+10000..10FFFF
N8 = {1: 0x80, 2: 0x800 - 0x80, 3: 0x10000 - 0x800 - 0x800, 4: 0x110000 - 0x10000}
#   UTF-16: one word for every non-surrogate, a pair for the supplementary planes
N16 = {1: 0x10000 - 0x800, 2: 0x110000 - 0x10000}


def valid_count(k, N, base):
    """Number of valid buffers of k units: V(k) = sum_L N_L V(k-L)."""
    V = [1]
    for j in range(1, k + 1):
        V.append(sum(N[L] * V[j - L] for L in N if L <= j))
    return V


def error_histogram(k, N, base):
    """Closed form: number of k-unit buffers whose first invalid character
    starts at p (the first p units form a valid buffer; the remaining k-p
    units do not begin with a complete valid character)."""
    V = valid_count(k, N, base)
    hist = {}
    for p in range(k):
        r = k - p
        not_start = base ** r - sum(N[L] * base ** (r - L) for L in N if L <= r)
        hist[p] = V[p] * not_start
    return V[k], hist


def cpy_utf8(b: bytes):
    try:
        s = b.decode("utf-8")
        return 0, len(b), s
    except UnicodeDecodeError as e:
        return -1, e.start, None


def cpy_utf16(b: bytes):
    try:
        s = b.decode("utf-16-le")
        return 0, len(b) // 2, s
    except UnicodeDecodeError as e:
        kind = O.UNPAIRED_LOW if e.reason == "illegal encoding" else O.UNPAIRED_HIGH
        return kind, e.start // 2, None


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

def test_closed_form_values():
    # sanity of the recurrences themselves (first terms)
    assert valid_count(4, N8, 256) == [1, 128, 18304, 2650112, 383270912]
    assert valid_count(2, N16, 65536) == [1, 63488, 4031774720]
    v, h = error_histogram(3, N8, 256)
    assert v + sum(h.values()) == 256 ** 3


@pytest.mark.parametrize("k", [1, 2, 3])
def test_all_utf8_buffers_closed_form(orc, k):
    """Every k-byte buffer: valid count and first-error histogram."""
    i = np.arange(256 ** k, dtype=np.uint32)
    cols = [((i >> (8 * (k - 1 - j))) & 0xFF).astype(np.uint8) for j in range(k)]
    data = np.stack(cols, axis=1).reshape(-1)
    offsets = np.arange(0, data.size + 1, k, dtype=np.int64)
    st, cnt = orc.validate_utf8_batch(data, offsets)
    v, hist = error_histogram(k, N8, 256)
    ok = st == 0
    assert int(ok.sum()) == v
    assert np.all(cnt[ok] == k)
    got = np.bincount(cnt[~ok].astype(np.int64), minlength=k)
    assert {p: int(got[p]) for p in range(k)} == hist
    # kinds are defined for every error
    assert set(np.unique(st[~ok]).tolist()) <= {1, 2, 3, 4, 5, 6}


def test_all_utf16_single_words(orc):
    data = np.arange(65536, dtype=np.uint16)
    offsets = np.arange(0, 65537, dtype=np.int64)
    st, cnt = orc.validate_utf16le_batch(data, offsets)
    assert int((st == 0).sum()) == N16[1]
    assert np.all(st[0xD800:0xDC00] == O.UNPAIRED_HIGH)
    assert np.all(st[0xDC00:0xE000] == O.UNPAIRED_LOW)


def test_utf16_pairs_closed_form_stratified(orc):
    """All 2-word buffers whose first word is any value and whose second word
    is drawn from every class boundary: compared with CPython, plus the
    closed-form count restricted to the sample (class products)."""
    second = np.array([0x0000, 0x0041, 0x007F, 0x0080, 0x07FF, 0x0800, 0xD7FF, 0xD800, 0xDA00,
                       0xDBFF, 0xDC00, 0xDD55, 0xDFFF, 0xE000, 0xFFFD, 0xFFFF], dtype=np.uint16)
    first = np.arange(65536, dtype=np.uint16)
    data = np.stack([np.repeat(first, second.size), np.tile(second, first.size)], axis=1).reshape(-1)
    offsets = np.arange(0, data.size + 1, 2, dtype=np.int64)
    st, cnt = orc.validate_utf16le_batch(data, offsets)
    # class-product closed form for the sample
    is_hi = lambda w: (w >= 0xD800) & (w <= 0xDBFF)
    is_lo = lambda w: (w >= 0xDC00) & (w <= 0xDFFF)
    nonsur = lambda w: ~(is_hi(w) | is_lo(w))
    expect_valid = int(nonsur(first).sum()) * int(nonsur(second).sum()) + \
        int(is_hi(first).sum()) * int(is_lo(second).sum())
    assert int((st == 0).sum()) == expect_valid
    # CPython on a seeded subset
    rng = np.random.default_rng(7)
    for j in rng.choice(st.size, size=20000, replace=False):
        b = data[2 * j:2 * j + 2].astype("<u2").tobytes()
        k, pos, _ = cpy_utf16(b)
        assert (int(st[j]), int(cnt[j]) if st[j] else 2) == ((k, pos) if k else (0, 2)), hex(data[2 * j])


# --------------------------------------------------------------------------
# exhaustive scalar values
# --------------------------------------------------------------------------

def _all_scalars():
    return np.concatenate([np.arange(0, 0xD800), np.arange(0xE000, 0x110000)]).astype(np.uint32)


def test_every_scalar_value_round_trips(orc):
    cps = _all_scalars()
    assert cps.size == 1112064
    s = cps.astype("<u4").tobytes().decode("utf-32-le")
    u8 = np.frombuffer(s.encode("utf-8"), dtype=np.uint8)
    u16 = np.frombuffer(s.encode("utf-16-le"), dtype="<u2")
    assert orc.validate_utf8(u8) == (0, u8.size)
    assert orc.validate_utf16le(u16) == (0, u16.size)
    assert orc.utf16_length_from_utf8(u8) == u16.size
    assert orc.utf8_length_from_utf16le(u16) == u8.size
    st, c, out = orc.convert_utf8_to_utf16le(u8, cap=u16.size)
    assert (st, c) == (0, u16.size) and np.array_equal(out, u16)
    st, c, out = orc.convert_utf16le_to_utf8(u16, cap=u8.size)
    assert (st, c) == (0, u8.size) and np.array_equal(out, u8)


def test_every_scalar_value_alone(orc):
    """Each scalar as its own string: valid, and its length by range
    (Section 3: 1 byte up to U+7F, 2 up to U+7FF, 3 up to U+FFFF, else 4)."""
    cps = _all_scalars()
    s = cps.astype("<u4").tobytes().decode("utf-32-le")
    u8 = np.frombuffer(s.encode("utf-8"), dtype=np.uint8)
    lens8 = np.where(cps < 0x80, 1, np.where(cps < 0x800, 2, np.where(cps < 0x10000, 3, 4)))
    off = np.zeros(cps.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens8)
    assert off[-1] == u8.size
    st, cnt = orc.validate_utf8_batch(u8, off)
    assert np.all(st == 0) and np.array_equal(cnt, lens8)
    st, cnt, out, oo = orc.convert_utf8_to_utf16le_batch(u8, off)
    assert np.all(st == 0)
    assert np.array_equal(np.diff(oo), np.where(cps < 0x10000, 1, 2))
    assert np.array_equal(out, np.frombuffer(s.encode("utf-16-le"), dtype="<u2"))


# --------------------------------------------------------------------------
# golden fixtures
# --------------------------------------------------------------------------

def _fixture(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append([f.strip() for f in line.split("|")])
    return rows


@pytest.mark.parametrize("row", _fixture("utf8_rules.txt"), ids=lambda r: r[0])
def test_golden_utf8(orc, row):
    data = np.array([int(x, 16) for x in row[0].split()], dtype=np.uint8)
    status, count = NAMES[row[1]], int(row[2])
    assert orc.validate_utf8(data) == (status, count)
    st, c, out = orc.convert_utf8_to_utf16le(data)
    if status == 0:
        words = [int(x, 16) for x in row[3].split()]
        assert (st, c) == (0, len(words)) and out[:c].tolist() == words
        assert orc.utf16_length_from_utf8(data) == len(words)
    else:
        assert (st, c) == (status, count)
    # CPython agrees on validity and position
    k, pos, _ = cpy_utf8(data.tobytes())
    assert (k == 0) == (status == 0) and pos == count


@pytest.mark.parametrize("row", _fixture("utf16_rules.txt"), ids=lambda r: r[0])
def test_golden_utf16(orc, row):
    data = np.array([int(x, 16) for x in row[0].split()], dtype=np.uint16)
    status, count = NAMES[row[1]], int(row[2])
    assert orc.validate_utf16le(data) == (status, count)
    st, c, out = orc.convert_utf16le_to_utf8(data)
    if status == 0:
        b = [int(x, 16) for x in row[3].split()]
        assert (st, c) == (0, len(b)) and out[:c].tolist() == b
        assert orc.utf8_length_from_utf16le(data) == len(b)
    else:
        assert (st, c) == (status, count)
    k, pos, _ = cpy_utf16(data.astype("<u2").tobytes())
    assert (k, pos) == ((status, count) if status else (0, data.size))


@pytest.mark.parametrize("row", _fixture("script_lengths.txt"), ids=lambda r: r[0])
def test_golden_script_lengths(orc, row):
    cp = int(row[1], 16)
    n8, n16 = int(row[2]), int(row[3])
    u16 = np.frombuffer(chr(cp).encode("utf-16-le"), dtype="<u2")
    assert u16.size * 2 == n16
    st, c, out = orc.convert_utf16le_to_utf8(u16)
    assert (st, c) == (0, n8)
    assert orc.utf16_length_from_utf8(out[:c]) * 2 == n16


# --------------------------------------------------------------------------
# CPython cross-checks on random inputs
# --------------------------------------------------------------------------

EDGE8 = np.array([0x00, 0x41, 0x7F, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC1, 0xC2, 0xDF,
                  0xE0, 0xE1, 0xEC, 0xED, 0xEE, 0xEF, 0xF0, 0xF1, 0xF3, 0xF4, 0xF5, 0xF7, 0xF8,
                  0xFF], dtype=np.uint8)


def _check_utf8_against_cpython(orc, b: bytes):
    arr = np.frombuffer(b, dtype=np.uint8)
    k, pos, s = cpy_utf8(b)
    st, cnt = orc.validate_utf8(arr)
    assert (st == 0) == (k == 0), b.hex()
    assert cnt == (len(b) if k == 0 else pos), b.hex()
    cst, cc, out = orc.convert_utf8_to_utf16le(arr)
    assert (cst, cc if cst else len(b)) == (st, cnt if st else len(b))
    if k == 0:
        ref = np.frombuffer(s.encode("utf-16-le"), dtype="<u2")
        assert cc == ref.size and np.array_equal(out[:cc], ref)
        assert orc.utf16_length_from_utf8(arr) == ref.size
    else:
        # output holds the conversion of the valid prefix
        ref = np.frombuffer(b[:pos].decode("utf-8").encode("utf-16-le"), dtype="<u2")
        assert np.array_equal(out[:ref.size], ref)


def test_random_edge_bytes_vs_cpython(orc):
    rng = np.random.default_rng(11)
    for _ in range(30000):
        n = int(rng.integers(1, 9))
        _check_utf8_against_cpython(orc, EDGE8[rng.integers(0, EDGE8.size, size=n)].tobytes())


def test_random_four_byte_buffers_vs_cpython(orc):
    """Seeded sample of 4-byte buffers, leads biased toward multi-byte."""
    rng = np.random.default_rng(12)
    lead = rng.integers(0xC0, 0x100, size=200000)
    rest = np.where(rng.random((200000, 3)) < 0.85, rng.integers(0x80, 0xC0, size=(200000, 3)),
                    rng.integers(0, 256, size=(200000, 3)))
    data = np.concatenate([lead[:, None], rest], axis=1).astype(np.uint8)
    offsets = np.arange(0, data.size + 1, 4, dtype=np.int64)
    st, cnt = orc.validate_utf8_batch(data.reshape(-1), offsets)
    for j in range(data.shape[0]):
        k, pos, _ = cpy_utf8(data[j].tobytes())
        assert (st[j] == 0) == (k == 0) and (cnt[j] if st[j] else 4) == (pos if k else 4), data[j].tobytes().hex()


def test_mutated_text_vs_cpython(orc):
    """Valid mixed text with random byte overwrites, deletions and cuts."""
    rng = np.random.default_rng(13)
    for it in range(3000):
        mix = ("mix1m",) + SCRIPT_MIXES
        t = random_text(rng, mix[it % len(mix)], int(rng.integers(1, 40)))
        b = bytearray(t.tobytes())
        for _ in range(int(rng.integers(0, 3))):
            op = int(rng.integers(0, 3))
            if not b:
                break
            p = int(rng.integers(0, len(b)))
            if op == 0:
                b[p] = int(EDGE8[rng.integers(0, EDGE8.size)])
            elif op == 1:
                del b[p]
            else:
                b = b[:p]
        if b:
            _check_utf8_against_cpython(orc, bytes(b))


def test_random_utf16_vs_cpython(orc):
    rng = np.random.default_rng(14)
    vals = np.array([0x0041, 0x00E9, 0x07FF, 0x0800, 0x4E2D, 0xD7FF, 0xD800, 0xDBFF, 0xDC00,
                     0xDFFF, 0xE000, 0xFFFF], dtype=np.uint16)
    for _ in range(30000):
        n = int(rng.integers(1, 8))
        w = vals[rng.integers(0, vals.size, size=n)]
        b = w.astype("<u2").tobytes()
        k, pos, s = cpy_utf16(b)
        assert O.validate_utf16le(w) == ((k, pos) if k else (0, n)), w
        st, c, out = orc.convert_utf16le_to_utf8(w)
        if k == 0:
            ref = s.encode("utf-8")
            assert st == 0 and out[:c].tobytes() == ref
            assert orc.utf8_length_from_utf16le(w) == len(ref)
        else:
            assert (st, c) == (k, pos)
            ref = b[:2 * pos].decode("utf-16-le").encode("utf-8")
            assert out[:len(ref)].tobytes() == ref


def _units16_of_utf8(b: bytes) -> int:
    """Reading 4 for UTF-8 input: one word per byte that is not a
    continuation byte (10xxxxxx), one more per byte >= F0."""
    a = np.frombuffer(b, dtype=np.uint8)
    return int(np.count_nonzero((a & 0xC0) != 0x80) + np.count_nonzero(a >= 0xF0))


def _units8_of_utf16(w: np.ndarray) -> int:
    """Reading 4 for UTF-16LE input: 1, 2 or 3 bytes per word by value
    (Section 3 ranges), 2 per surrogate word."""
    w = w.astype(np.int64)
    sur = (w >= 0xD800) & (w <= 0xDFFF)
    return int(np.sum(np.where(w < 0x80, 1, np.where(w < 0x800, 2, np.where(sur, 2, 3)))))


def _edit16(rng, w):
    """Overwrite, delete or cut one word, biased toward surrogates."""
    w = list(w)
    if not w:
        return w
    p, op = int(rng.integers(0, len(w))), int(rng.integers(0, 3))
    if op == 0:
        w[p] = int(rng.choice([0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0x0041, 0x20AC]))
    elif op == 1:
        del w[p]
    else:
        w = w[:p]
    return w


def test_batch_conversions_vs_cpython_per_string(orc):
    """Reading 9: in one batched call each string is converted as if alone
    (status and position as CPython's strict codec finds them for that
    string alone, exact output for a valid string) and its output starts at
    the sum of the reading-4 lengths of the strings before it."""
    rng = np.random.default_rng(15)
    mixes = ("mix1m",) + SCRIPT_MIXES
    for rep in range(40):
        k = int(rng.integers(1, 60))
        s8, s16 = [], []
        for i in range(k):
            t = random_text(rng, mixes[(rep + i) % len(mixes)], int(rng.integers(0, 30)))
            b = bytearray(t.tobytes())
            if b and rng.random() < 0.3:   # an invalid string: one byte edited, deleted or cut
                p, op = int(rng.integers(0, len(b))), int(rng.integers(0, 3))
                if op == 0:
                    b[p] = int(EDGE8[rng.integers(0, EDGE8.size)])
                elif op == 1:
                    del b[p]
                else:
                    b = b[:p]
            s8.append(bytes(b))
            w = np.frombuffer(t.tobytes().decode("utf-8").encode("utf-16-le"), dtype="<u2")
            if w.size and rng.random() < 0.3:
                w = np.array(_edit16(rng, w), dtype=np.uint16)
            s16.append(np.asarray(w, dtype=np.uint16))
        # UTF-8 -> UTF-16LE
        data = np.frombuffer(b"".join(s8) or b"\0", dtype=np.uint8)[:sum(map(len, s8))]
        off = np.concatenate([[0], np.cumsum([len(x) for x in s8])]).astype(np.int64)
        st, cnt, out, oo = orc.convert_utf8_to_utf16le_batch(data, off)
        assert np.array_equal(oo, np.concatenate([[0], np.cumsum([_units16_of_utf8(x) for x in s8])]))
        for i, x in enumerate(s8):
            kind, pos, txt = cpy_utf8(x)
            assert (st[i] == 0) == (kind == 0), (rep, i, x.hex())
            if kind == 0:
                ref = np.frombuffer(txt.encode("utf-16-le"), dtype="<u2")
                assert cnt[i] == ref.size and np.array_equal(out[oo[i]:oo[i] + ref.size], ref), (rep, i)
            else:
                assert cnt[i] == pos, (rep, i, x.hex())
        # UTF-16LE -> UTF-8
        d16 = np.concatenate(s16).astype(np.uint16) if k else np.zeros(0, np.uint16)
        off16 = np.concatenate([[0], np.cumsum([x.size for x in s16])]).astype(np.int64)
        st, cnt, out, oo = orc.convert_utf16le_to_utf8_batch(d16, off16)
        assert np.array_equal(oo, np.concatenate([[0], np.cumsum([_units8_of_utf16(x) for x in s16])]))
        for i, x in enumerate(s16):
            kind, pos, txt = cpy_utf16(x.astype("<u2").tobytes())
            assert (st[i], cnt[i]) == ((0, len(txt.encode("utf-8"))) if kind == 0 else (kind, pos)), (rep, i, x)
            if kind == 0:
                ref = np.frombuffer(txt.encode("utf-8"), dtype=np.uint8)
                assert np.array_equal(out[oo[i]:oo[i] + ref.size], ref), (rep, i)


# --------------------------------------------------------------------------
# invariants on generated text
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mix", ("mix1m",) + SCRIPT_MIXES)
def test_round_trip_and_lengths(orc, mix):
    rng = np.random.default_rng(21)
    u8 = random_text(rng, mix, 20000)
    n16 = orc.utf16_length_from_utf8(u8)
    st, c, u16 = orc.convert_utf8_to_utf16le(u8, cap=n16)
    assert (st, c) == (0, n16)
    n8 = orc.utf8_length_from_utf16le(u16)
    assert n8 == u8.size
    st, c, back = orc.convert_utf16le_to_utf8(u16, cap=n8)
    assert (st, c) == (0, u8.size) and np.array_equal(back, u8)


def test_concatenation_and_prefix(orc):
    rng = np.random.default_rng(22)
    for _ in range(200):
        a = random_text(rng, "mix1m", int(rng.integers(0, 50)))
        b = random_text(rng, "emoji", int(rng.integers(0, 50)))
        ab = np.concatenate([a, b])
        _, ca, oa = orc.convert_utf8_to_utf16le(a)
        _, cb, ob = orc.convert_utf8_to_utf16le(b)
        st, cab, oab = orc.convert_utf8_to_utf16le(ab)
        assert st == 0 and np.array_equal(oab[:cab], np.concatenate([oa[:ca], ob[:cb]]))
        # prefix property: cut anywhere, the first error (if any) leaves a valid prefix
        cut = int(rng.integers(0, ab.size + 1))
        st, e = orc.validate_utf8(ab[:cut])
        if st:
            assert e < cut and orc.validate_utf8(ab[:e]) == (0, e)


def test_output_too_small(orc):
    u8 = np.frombuffer("aé中😀".encode(), dtype=np.uint8)
    st, c, out = orc.convert_utf8_to_utf16le(u8, cap=3)
    assert (st, c) == (O.OUTPUT_TOO_SMALL, 5)
    assert out.tolist() == [0x61, 0xE9, 0x4E2D]
    u16 = np.frombuffer("aé中😀".encode("utf-16-le"), dtype="<u2")
    st, c, out = orc.convert_utf16le_to_utf8(u16, cap=4)
    assert (st, c) == (O.OUTPUT_TOO_SMALL, 10)
    assert out.tobytes() == "aé中".encode()[:4]
    # a data error takes precedence over the capacity
    bad = np.frombuffer(b"abc\x80", dtype=np.uint8)
    st, c, _ = orc.convert_utf8_to_utf16le(bad, cap=1)
    assert (st, c) == (O.TOO_LONG, 3)


def test_empty(orc):
    e8 = np.zeros(0, dtype=np.uint8)
    e16 = np.zeros(0, dtype=np.uint16)
    assert orc.validate_utf8(e8) == (0, 0)
    assert orc.validate_utf16le(e16) == (0, 0)
    assert orc.utf16_length_from_utf8(e8) == 0
    assert orc.utf8_length_from_utf16le(e16) == 0
    assert orc.convert_utf8_to_utf16le(e8, cap=0)[:2] == (0, 0)
    assert orc.convert_utf16le_to_utf8(e16, cap=0)[:2] == (0, 0)
