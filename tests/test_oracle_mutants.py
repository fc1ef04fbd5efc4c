"""Pin strength: plausible mistakes planted in copies of the oracle source
(on the CPU) must each be caught by at least one independent pin.

Each mutant is compiled from a textually edited copy of
``oracle/utf_oracle.c`` into a temporary directory and run through a
compact battery of the checks in ``test_oracle_pins.py`` (closed forms,
exhaustive scalars, golden fixtures, CPython cross-checks).  The unmodified
source must pass the battery.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
from tests.test_oracle_pins import (EDGE8, N8, _all_scalars, _edit16, _fixture, _units8_of_utf16,
                                    _units16_of_utf8, cpy_utf8, cpy_utf16, error_histogram)
from workloads import random_text

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "utf_oracle.c")
NAMES = {v: k for k, v in O.STATUS_NAMES.items()}

# (description, exact text, replacement); the first occurrence is replaced
MUTANTS = [
    ("two-byte payload mask", "cp = lead & 0x1F;", "cp = lead & 0x0F;"),
    ("three-byte payload mask", "cp = lead & 0x0F;", "cp = lead & 0x07;"),
    ("four-byte payload mask", "cp = lead & 0x07;", "cp = lead & 0x03;"),
    ("continuation shift", "cp = (cp << 6) |", "cp = (cp << 5) |"),
    ("continuation payload", "(uint32_t)(s[i + k] & 0x3F)", "(uint32_t)(s[i + k] & 0x1F)"),
    ("continuation test", "if ((s[i + k] & 0xC0) != 0x80)", "if ((s[i + k] & 0x80) != 0x80)"),
    ("rule 1 mask", "(lead & 0xF8) == 0xF8", "(lead & 0xFC) == 0xFC"),
    ("rule 3 test", "(lead & 0xC0) == 0x80", "(lead & 0xE0) == 0x80"),
    ("two-byte lead pattern", "(lead & 0xE0) == 0xC0", "(lead & 0xC0) == 0xC0"),
    ("rule 4, 2 bytes", "len == 2 && cp <= 0x7F", "len == 2 && cp < 0x7F"),
    ("rule 4, 3 bytes", "len == 3 && cp <= 0x7FF", "len == 3 && cp <= 0x7F"),
    ("rule 4, 4 bytes", "len == 4 && cp <= 0xFFFF", "len == 4 && cp <= 0xFFF"),
    ("rule 5 bound", "cp >= 1114112", "cp > 1114112"),
    ("rule 6 upper", "cp >= 0xD800 && cp <= 0xDFFF", "cp >= 0xD800 && cp < 0xDFFF"),
    ("rule 6 lower", "cp >= 0xD800 && cp <= 0xDFFF", "cp > 0xD800 && cp <= 0xDFFF"),
    ("kind swap overlong", "return OR_OVERLONG;", "return OR_TOO_LARGE;"),
    ("kind swap too short", "return OR_TOO_SHORT;", "return OR_TOO_LONG;"),
    ("first error offset", "r.count = i;\n            return r;", "r.count = i + 1;\n            return r;"),
    ("utf16 pair shift", "(((w & 0x3FF) << 10)", "(((w & 0x3FF) << 9)"),
    ("utf16 pair offset", "*cp_out = 0x10000 +", "*cp_out = 0x1000 +"),
    ("utf16 low bound", "if (w >= 0xDC00)\n        return OR_UNPAIRED_LOW;", "if (w > 0xDC00)\n        return OR_UNPAIRED_LOW;"),
    ("utf16 second word", "if (w2 < 0xDC00 || w2 > 0xDFFF)", "if (w2 < 0xDC00 || w2 >= 0xDFFF)"),
    ("utf16 encode high", "0xD800 | (v >> 10)", "0xD800 | (v >> 11)"),
    ("utf16 encode low", "0xDC00 | (v & 0x3FF)", "0xDC00 | (v & 0x1FF)"),
    ("utf16 encode bound", "if (cp < 0x10000) {\n        w[0]", "if (cp <= 0x10000) {\n        w[0]"),
    ("utf8 encode 2-byte lead", "0xC0 | (cp >> 6)", "0xC0 | (cp >> 5)"),
    ("utf8 encode range", "if (cp <= 0x7FF) {", "if (cp < 0x7FF) {"),
    ("utf8 encode 3-byte middle", "0x80 | ((cp >> 6) & 0x3F));\n        b[2]", "0x80 | ((cp >> 5) & 0x3F));\n        b[2]"),
    ("utf8 encode 4-byte lead", "0xF0 | (cp >> 18)", "0xF0 | (cp >> 17)"),
    ("utf8 encode 4-byte second", "0x80 | ((cp >> 12) & 0x3F));\n    b[2]", "0x80 | ((cp >> 12) & 0x1F));\n    b[2]"),
    ("length: pair test", "if (b >= 0xF0)\n            words += 1;", "if (b > 0xF0)\n            words += 1;"),
    ("length: continuation test", "if ((b & 0xC0) == 0x80)\n            continue;", "if ((b & 0xE0) == 0x80)\n            continue;"),
    ("length: two-byte bound", "else if (w <= 0x7FF)\n            bytes += 2;", "else if (w < 0x7FF)\n            bytes += 2;"),
    ("length: surrogate words", "else if (w >= 0xD800 && w <= 0xDFFF)\n            bytes += 2;", "else if (w >= 0xD800 && w <= 0xDFFF)\n            bytes += 3;"),
    ("capacity test", "if (o > cap) {", "if (o >= cap) {"),
    ("word assembly", "((uint32_t)s[2 * i + 1] << 8)", "((uint32_t)s[2 * i + 1] << 7)"),
    # batched forms (each keeps every write inside the output the wrapper sizes)
    ("utf-8 batch output offsets", "out + 2 * o, room);\n        o += (int64_t)room;",
     "out + 2 * o, room);\n        o += (int64_t)(room ? room - 1 : 0);"),
    ("utf-16 batch output offsets", "out + o, room);\n        o += (int64_t)room;",
     "out + o, room);\n        o += (int64_t)len;"),
    ("utf-16 batch reported offset", "out_offsets[j] = o;\n        results[j] = oracle_convert_utf16le_to_utf8",
     "out_offsets[j] = o + (j > 0);\n        results[j] = oracle_convert_utf16le_to_utf8"),
]


def battery(lib) -> list:
    """Returns the names of the checks that fail with ``lib``."""
    failed = []

    def check(name, fn):
        try:
            if not fn():
                failed.append(name)
        except AssertionError:
            failed.append(name)

    def closed_form(k):
        i = np.arange(256 ** k, dtype=np.uint32)
        data = np.stack([((i >> (8 * (k - 1 - j))) & 0xFF).astype(np.uint8) for j in range(k)], 1).reshape(-1)
        st, cnt = O.validate_utf8_batch(data, np.arange(0, data.size + 1, k, dtype=np.int64), lib=lib)
        v, hist = error_histogram(k, N8, 256)
        ok = st == 0
        got = np.bincount(cnt[~ok].astype(np.int64), minlength=k)
        return int(ok.sum()) == v and {p: int(got[p]) for p in range(k)} == hist

    def scalars():
        s = _all_scalars().astype("<u4").tobytes().decode("utf-32-le")
        u8 = np.frombuffer(s.encode("utf-8"), dtype=np.uint8)
        u16 = np.frombuffer(s.encode("utf-16-le"), dtype="<u2")
        a = O.convert_utf8_to_utf16le(u8, cap=u16.size, lib=lib)
        b = O.convert_utf16le_to_utf8(u16, cap=u8.size, lib=lib)
        return (a[:2] == (0, u16.size) and np.array_equal(a[2], u16)
                and b[:2] == (0, u8.size) and np.array_equal(b[2], u8)
                and O.utf16_length_from_utf8(u8, lib=lib) == u16.size
                and O.utf8_length_from_utf16le(u16, lib=lib) == u8.size)

    def golden():
        for row in _fixture("utf8_rules.txt"):
            d = np.array([int(x, 16) for x in row[0].split()], dtype=np.uint8)
            if O.validate_utf8(d, lib=lib) != (NAMES[row[1]], int(row[2])):
                return False
            st, c, out = O.convert_utf8_to_utf16le(d, lib=lib)
            if NAMES[row[1]] == 0 and out[:c].tolist() != [int(x, 16) for x in row[3].split()]:
                return False
        for row in _fixture("utf16_rules.txt"):
            d = np.array([int(x, 16) for x in row[0].split()], dtype=np.uint16)
            if O.validate_utf16le(d, lib=lib) != (NAMES[row[1]], int(row[2])):
                return False
            st, c, out = O.convert_utf16le_to_utf8(d, lib=lib)
            if NAMES[row[1]] == 0 and out[:c].tolist() != [int(x, 16) for x in row[3].split()]:
                return False
        return True

    def cpython8():
        rng = np.random.default_rng(11)
        for _ in range(3000):
            b = EDGE8[rng.integers(0, EDGE8.size, size=int(rng.integers(1, 9)))].tobytes()
            k, pos, s = cpy_utf8(b)
            arr = np.frombuffer(b, dtype=np.uint8)
            st, cnt = O.validate_utf8(arr, lib=lib)
            if (st == 0) != (k == 0) or cnt != (len(b) if k == 0 else pos):
                return False
            if k == 0 and O.utf16_length_from_utf8(arr, lib=lib) != len(s.encode("utf-16-le")) // 2:
                return False
        return True

    def cpython16():
        rng = np.random.default_rng(14)
        vals = np.array([0x41, 0xE9, 0x7FF, 0x800, 0x4E2D, 0xD7FF, 0xD800, 0xDBFF, 0xDC00, 0xDFFF,
                         0xE000, 0xFFFF], dtype=np.uint16)
        for _ in range(3000):
            w = vals[rng.integers(0, vals.size, size=int(rng.integers(1, 8)))]
            k, pos, s = cpy_utf16(w.astype("<u2").tobytes())
            if O.validate_utf16le(w, lib=lib) != ((k, pos) if k else (0, w.size)):
                return False
            if k == 0 and O.utf8_length_from_utf16le(w, lib=lib) != len(s.encode("utf-8")):
                return False
        return True

    def capacity():
        u8 = np.frombuffer("aé中😀".encode(), dtype=np.uint8)
        r1 = O.convert_utf8_to_utf16le(u8, cap=5, lib=lib)[:2] == (0, 5)
        r2 = O.convert_utf8_to_utf16le(u8, cap=4, lib=lib)[:2] == (O.OUTPUT_TOO_SMALL, 5)
        return r1 and r2

    check("closed form k=2", lambda: closed_form(2))
    check("closed form k=3", lambda: closed_form(3))
    check("scalar round trip", scalars)
    check("golden", golden)
    check("cpython utf-8", cpython8)
    check("cpython utf-16", cpython16)
    def batches():
        rng = np.random.default_rng(16)
        for _ in range(20):
            k = int(rng.integers(1, 30))
            s8 = [random_text(rng, "mix1m", int(rng.integers(0, 20))).tobytes() for _ in range(k)]
            s16 = []
            for x in s8:
                w = np.frombuffer(x.decode("utf-8").encode("utf-16-le"), dtype="<u2").astype(np.uint16)
                s16.append(np.array(_edit16(rng, w), dtype=np.uint16) if w.size and rng.random() < 0.3 else w)
            data = np.frombuffer(b"".join(s8) + b"\0", dtype=np.uint8)[:sum(map(len, s8))]
            off = np.concatenate([[0], np.cumsum([len(x) for x in s8])]).astype(np.int64)
            st, cnt, out, oo = O.convert_utf8_to_utf16le_batch(data, off, lib=lib)
            if not np.array_equal(oo, np.concatenate([[0], np.cumsum([_units16_of_utf8(x) for x in s8])])):
                return False
            for i, x in enumerate(s8):
                ref = np.frombuffer(x.decode("utf-8").encode("utf-16-le"), dtype="<u2")
                if st[i] != 0 or cnt[i] != ref.size or not np.array_equal(out[oo[i]:oo[i] + ref.size], ref):
                    return False
            d16 = np.concatenate(s16 + [np.zeros(1, np.uint16)])[:sum(x.size for x in s16)]
            off16 = np.concatenate([[0], np.cumsum([x.size for x in s16])]).astype(np.int64)
            st, cnt, out, oo = O.convert_utf16le_to_utf8_batch(d16, off16, lib=lib)
            if not np.array_equal(oo, np.concatenate([[0], np.cumsum([_units8_of_utf16(x) for x in s16])])):
                return False
            for i, x in enumerate(s16):
                kind, pos, txt = cpy_utf16(x.astype("<u2").tobytes())
                if (st[i], cnt[i]) != ((0, len(txt.encode("utf-8"))) if kind == 0 else (kind, pos)):
                    return False
                ref = np.frombuffer(txt.encode("utf-8"), dtype=np.uint8) if kind == 0 else None
                if ref is not None and not np.array_equal(out[oo[i]:oo[i] + ref.size], ref):
                    return False
        return True

    check("capacity", capacity)
    check("batches", batches)
    return failed


def _compile(src_text, tmpdir, tag):
    c = os.path.join(tmpdir, f"m_{tag}.c")
    so = os.path.join(tmpdir, f"m_{tag}.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", c, "-o", so])
    return O.load(so)


@pytest.fixture(scope="module")
def tmpdir_mut():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_unmodified_oracle_passes_battery(tmpdir_mut):
    lib = _compile(open(SRC).read(), tmpdir_mut, "orig")
    assert battery(lib) == []


@pytest.mark.parametrize("desc,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmpdir_mut, desc, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    mutated = src.replace(old, new, 1)
    lib = _compile(mutated, tmpdir_mut, str(abs(hash(desc))))
    failed = battery(lib)
    assert failed, f"mutant '{desc}' survived every pin"
