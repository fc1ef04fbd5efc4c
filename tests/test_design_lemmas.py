"""CPU checks of the two facts the GPU kernels rest on, against the oracle.

1. Locality.  The greedy first error equals the smallest position i at which
   a predicate C(i) over the window b[i-3..i+3] holds:
     * b_i not a continuation: the character announced at i breaks a rule
       of Section 3 (bytes past the end count as missing);
     * b_i a continuation: no j in {i-1, i-2, i-3} has b_j >= 0xC0
       announcing more than i-j bytes with only continuations in between.
   For UTF-16: a high word not followed by a low word, or a low word not
   preceded by a high word.
2. Detection.  Let must(t) = [b_{t-1} >= C0] | [b_{t-2} >= E0] |
   [b_{t-3} >= F0] and cont(t) = [b_t in 80..BF].  For the first error e,
   either must(t) != cont(t) for some t in [e, e+3] (bytes past the end
   read as 0x00), or the character at e is structurally complete and its
   decoded value breaks rule 4, 5 or 6 (or its lead breaks rule 1).  The
   kernels therefore only run the exact per-position scan on waves where
   one of those cheap signals fired.
3. Per-wave control.  A wave owning positions [a, z) computes its byte
   class over [a-3, z) (the three bytes before it included); with no byte
   >= 0xF0 it drops the F0 term of must(), with no byte >= 0xE0 also the E0
   term, and with no byte >= 0x80 it raises nothing.  It flags when a
   mismatch occurs at one of its positions or a value rule fails at one of
   its leading bytes, and a flagged wave evaluates C exactly over its own
   positions [a, z) and over the non-continuation positions of [a-3, a)
   (a continuation byte there is judged by the wave that owns it, whose
   detector fires at that very byte when it is the first error).
   Splitting a buffer into waves at any point, the smallest C found this
   way is the greedy first error.
"""
import itertools

import numpy as np
import pytest

import oracle as O

ALPHA = [0x41, 0x80, 0x8F, 0x90, 0x9F, 0xA0, 0xBF, 0xC0, 0xC2, 0xDF, 0xE0, 0xE1, 0xED, 0xEF,
         0xF0, 0xF4, 0xF5, 0xF8]


def is_cont(x):
    return 0x80 <= x <= 0xBF


def announced(x):
    return 1 if x < 0x80 else 2 if x < 0xE0 else 3 if x < 0xF0 else 4


def char_fails(b, i):
    """Rules 1-6 for the character announced at a non-continuation b[i]."""
    x = b[i]
    if x < 0x80:
        return False
    if x >= 0xF8:
        return True
    L = announced(x)
    for k in range(1, L):
        if i + k >= len(b) or not is_cont(b[i + k]):
            return True
    cp = x & (0x7F >> L)
    for k in range(1, L):
        cp = (cp << 6) | (b[i + k] & 0x3F)
    lo = {2: 0x80, 3: 0x800, 4: 0x10000}[L]
    return cp < lo or cp > 0x10FFFF or 0xD800 <= cp <= 0xDFFF


def C(b, i):
    if not is_cont(b[i]):
        return char_fails(b, i)
    for d in (1, 2, 3):
        j = i - d
        if j < 0:
            break
        if b[j] >= 0xC0 and announced(b[j]) > d and all(is_cont(b[t]) for t in range(j + 1, i)):
            return False
    return True


def byte_at(b, t):
    return b[t] if 0 <= t < len(b) else 0x00


def must(b, t, terms=3):
    m = byte_at(b, t - 1) >= 0xC0
    if terms >= 2:
        m = m or byte_at(b, t - 2) >= 0xE0
    if terms >= 3:
        m = m or byte_at(b, t - 3) >= 0xF0
    return m


def range_flag(b, i):
    """Value rules (and rule 1) at a non-continuation byte whose announced
    continuation bytes are all present."""
    x = b[i]
    if x < 0x80 or is_cont(x):
        return False
    if x >= 0xF8:
        return True
    L = announced(x)
    if any(not is_cont(byte_at(b, i + k)) for k in range(1, L)) or i + L > len(b):
        return False
    return char_fails(b, i)


def check_buffer(b):
    st, e = O.validate_utf8(np.array(b, dtype=np.uint8))
    cs = [i for i in range(len(b)) if C(b, i)]
    if st == 0:
        assert not cs, bytes(b).hex()
        return
    assert cs and cs[0] == e, (bytes(b).hex(), cs, e)
    # detection
    mis = any(must(b, t) != is_cont(byte_at(b, t)) for t in range(e, e + 4))
    assert mis or range_flag(b, e), bytes(b).hex()
    # narrowed detectors when no byte >= F0 (or >= E0) occurs at or after e's window
    for terms, bound in ((2, 0xF0), (1, 0xE0)):
        if all(x < bound for x in b):
            mis = any(must(b, t, terms) != is_cont(byte_at(b, t)) for t in range(e, e + 4))
            assert mis or range_flag(b, e), (terms, bytes(b).hex())


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_locality_and_detection_exhaustive(n):
    for b in itertools.product(ALPHA, repeat=n):
        check_buffer(list(b))


def test_locality_and_detection_random_long():
    rng = np.random.default_rng(5)
    alpha = np.array(ALPHA + [0x20, 0x7F, 0xBE, 0xE4, 0xB8, 0xF1, 0xF3], dtype=np.uint8)
    for _ in range(40000):
        n = int(rng.integers(5, 12))
        check_buffer(alpha[rng.integers(0, alpha.size, size=n)].tolist())


def test_utf16_locality_exhaustive():
    W = [0x0041, 0xD800, 0xDBFF, 0xDC00, 0xDFFF, 0xE000]
    for n in range(1, 6):
        for w in itertools.product(W, repeat=n):
            st, e = O.validate_utf16le(np.array(w, dtype=np.uint16))
            hi = [0xD800 <= x <= 0xDBFF for x in w]
            lo = [0xDC00 <= x <= 0xDFFF for x in w]
            cs = [i for i in range(n)
                  if (hi[i] and (i + 1 >= n or not lo[i + 1])) or (lo[i] and (i == 0 or not hi[i - 1]))]
            if st == 0:
                assert not cs
            else:
                assert cs[0] == e


def wave_class(b, lo, hi):
    seg = [b[t] for t in range(max(lo, 0), min(hi, len(b)))]
    top = max(seg) if seg else 0
    return 0 if top < 0x80 else 1 if top < 0xE0 else 2 if top < 0xF0 else 3


def wave_found(b, a, z):
    """Model of one wave: returns the exact C positions it reports, or []."""
    n = len(b)
    cls = wave_class(b, a - 3, z)
    if cls == 0:
        return []
    terms = cls
    flag = any(must(b, t, terms) != is_cont(byte_at(b, t)) for t in range(a, z))
    flag = flag or any(range_flag(b, i) for i in range(max(a, 0), min(z, n)))
    if not flag:
        return []
    halo = [i for i in range(max(a - 3, 0), min(a, n)) if not is_cont(b[i]) and C(b, i)]
    return halo + [i for i in range(max(a, 0), min(z, n)) if C(b, i)]


def check_split(b):
    n = len(b)
    st, e = O.validate_utf8(np.array(b, dtype=np.uint8))
    for cut in range(0, n + 1):
        waves = [(0, cut), (cut, n + 3)] if cut > 0 else [(0, n + 3)]
        found = [i for a, z in waves for i in wave_found(b, a, z)]
        if st == 0:
            assert not found, bytes(b).hex()
        else:
            assert found and min(found) == e, (bytes(b).hex(), cut, found, e)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_wave_control_exhaustive(n):
    alpha = [0x41, 0x80, 0x9F, 0xA0, 0xBF, 0xC0, 0xC2, 0xE0, 0xE4, 0xED, 0xF0, 0xF4, 0xF5, 0xF8]
    for b in itertools.product(alpha, repeat=n):
        check_split(list(b))


def test_wave_control_random_long():
    rng = np.random.default_rng(6)
    alpha = np.array(ALPHA + [0x20, 0x7F, 0xBE, 0xE4, 0xB8, 0xF1, 0xF3], dtype=np.uint8)
    for _ in range(6000):
        n = int(rng.integers(5, 14))
        check_split(alpha[rng.integers(0, alpha.size, size=n)].tolist())


# 4. Exact first error from three byte-local flags.  A flagged wave finds
#    its first error as the first position carrying one of: a continuation
#    byte with must() false, a leading byte whose announced continuation
#    bytes are not all continuations, a leading byte whose (lead, next byte)
#    pair breaks a value rule (C0/C1; E0 80..9F; ED A0..BF; F0 80..8F;
#    F4 90..BF; F5..FF).  Every flag implies C at its position and the first
#    position of C carries a flag, so the first flag is the first error.

def flags_at(b, i):
    x = byte_at(b, i)
    nxt = byte_at(b, i + 1)
    if is_cont(x):
        return not must(b, i)
    if x < 0xC0:
        return False
    L = announced(x)
    if any(not is_cont(byte_at(b, i + k)) for k in range(1, L)):
        return True
    return (x in (0xC0, 0xC1) or (x == 0xE0 and nxt < 0xA0) or (x == 0xED and nxt >= 0xA0)
            or (x == 0xF0 and nxt < 0x90) or (x == 0xF4 and nxt >= 0x90) or x >= 0xF5)


def check_first_flag(b):
    st, e = O.validate_utf8(np.array(b, dtype=np.uint8))
    fl = [i for i in range(len(b)) if flags_at(b, i)]
    if st == 0:
        assert not fl, bytes(b).hex()
    else:
        assert fl and fl[0] == e, (bytes(b).hex(), fl, e)
        assert all(C(b, i) for i in fl), bytes(b).hex()


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_first_flag_exhaustive(n):
    for b in itertools.product(ALPHA, repeat=n):
        check_first_flag(list(b))


def test_first_flag_random_long():
    rng = np.random.default_rng(9)
    alpha = np.array(ALPHA + [0x20, 0x7F, 0xBE, 0xE4, 0xB8, 0xF1, 0xF3], dtype=np.uint8)
    for _ in range(30000):
        n = int(rng.integers(5, 14))
        check_first_flag(alpha[rng.integers(0, alpha.size, size=n)].tolist())


# 5. Slot write order of the UTF-8 -> UTF-16 scatter.  Per row, lane L
#    holds bytes 16L..16L+15; its first slot is the exclusive prefix of
#    the lanes' slot counts (one per non-continuation byte, one more per
#    byte >= F0 when the wave has one).  Instruction k (k = 0..15) has every
#    lane store the window of its byte k at the slot of its next leading
#    byte (and, with bytes >= F0 about, a marked copy first: at the next
#    slot for a byte >= F0, else at the same slot).  Afterwards each lane
#    rewrites its first slot with its first leading byte's window (waves in
#    the middle of the input only look in the chunk's first dword).  The
#    slots of every character before the first error must hold that
#    character's window, whatever order the lanes of one instruction take.

def scatter_model(row, lo, hi, kany, lane_order, edge):
    b = [row[i] if lo <= i < hi else 0 for i in range(len(row))]
    lead = [lo <= i < hi and not is_cont(b[i]) for i in range(1024)]
    f0 = [kany and b[i] >= 0xF0 for i in range(1024)]
    width = [sum(int(lead[16 * L + k]) + int(f0[16 * L + k]) for k in range(16)) for L in range(64)]
    base = [sum(width[:L]) for L in range(64)]
    last = 1032 - 2
    o = list(base)
    stage = {}
    win = lambda i: b[i] | b[i + 1] << 8 | b[i + 2] << 16 | b[i + 3] << 24
    for k in range(16):
        marked, plain = [], []
        for L in range(64):
            i = 16 * L + k
            a = min(o[L], last) if kany else o[L]
            if kany:
                marked.append((L, a + int(f0[i]), win(i) ^ 0x70))
            plain.append((L, a, win(i)))
            o[L] += int(lead[i]) + int(f0[i])
        for group in (marked, plain):
            for L, a, v in sorted(group, reverse=(lane_order == "high")):
                assert a < 1032
                stage[a] = v
    for L in range(64):
        first = [k for k in range(16) if lead[16 * L + k]]
        if not first or (not edge and first[0] > 3):
            continue
        stage[min(base[L], last) if kany else base[L]] = win(16 * L + first[0])
    return stage, lead, f0, win


def check_scatter(row, lo, hi, valid_upto):
    kany = any(x >= 0xF0 for x in row[max(lo - 3, 0):hi])
    edge = lo > 0 or hi < len(row)
    for order in ("low", "high"):
        stage, lead, f0, win = scatter_model(row, lo, hi, kany, order, edge)
        s = 0
        for i in range(valid_upto):
            if lead[i]:
                assert stage.get(s) == win(i), (order, i, s)
                s += 1
                if f0[i]:
                    assert stage.get(s) == win(i) ^ 0x70, (order, i, s)
                    s += 1


def test_scatter_write_order():
    from workloads import random_text, SCRIPT_MIXES
    rng = np.random.default_rng(11)
    mixes = ("mix1m",) + tuple(SCRIPT_MIXES)
    for trial in range(48):
        t = np.frombuffer(random_text(rng, mixes[trial % len(mixes)], 1200), dtype=np.uint8)
        start = int(rng.integers(0, 4))
        row = [int(x) for x in t[start:start + 1028]]
        lo = 0 if trial % 3 else int(rng.integers(0, 40))
        hi = 1028 if trial % 4 else int(rng.integers(900, 1028))
        e = 1024
        if trial % 2:   # an injected error: only the slots before it must hold
            e = int(rng.integers(0, 1020))
            kind = (trial // 2) % 4
            if kind == 0:
                row[e] = 0x80
            elif kind == 1:
                row[e] = 0xF8
            elif kind == 2:
                row[e:e + 8] = [0xF1] * 8
            else:
                row[e:e + 20] = [0x80] * 20
            row = row[:1028]
        check_scatter(row, lo, hi, max(min(e, hi) - 4, 0))


# 5. Write order of the packed path for waves of ASCII and four-byte
#    characters (scatter_quad): in instruction k, every lane stores the
#    first word of its position k (the byte, or the high surrogate of the
#    character starting there) at the slot of its next leading byte and the
#    low surrogate at the slot after; lanes of one instruction may land in
#    any order.  Then each lane rewrites its first two slots: its first
#    character's first word, then that character's low surrogate or the
#    next character's first word.  Every slot of a valid row must hold the
#    character's word, for both lane orders.  The words are computed here
#    from the characters themselves (chr / encode), not from the kernel's
#    packed formulas, so the formulas are checked too.

def quad_words_at(b, q):
    """(first word, low surrogate) the kernel computes at position q:
    packed 16-bit formulas for a leading byte >= F0, the byte otherwise."""
    a, bb, c, d = b[q], b[q + 1], b[q + 2], b[q + 3]
    first = ((a * 256 + bb * 4 + (c >> 4) + 0xE5B8) & 0xFFFF) if a >= 0xF0 else a
    low = ((c & 0x0F) * 64 + d + 0xDB80) & 0xFFFF
    return first, low


def test_quad_write_order():
    rng = np.random.default_rng(12)
    for trial in range(40):
        cps = []
        data = b""
        while len(data) < 1024 + 16:
            cp = int(rng.integers(0x20, 0x7F)) if rng.random() < 0.7 else int(rng.integers(0x10000, 0x110000))
            cps.append(cp)
            data += chr(cp).encode("utf-8")
        b = list(data) + [0] * 8
        lead = [(x & 0xC0) != 0x80 for x in b]
        width = [int(lead[i]) + int(b[i] >= 0xF0) for i in range(len(b))]
        lw = [sum(width[16 * L:16 * L + 16]) for L in range(64)]
        base = [sum(lw[:L]) for L in range(64)]
        for order in ("low", "high"):
            o = list(base)
            stage = {}
            for k in range(16):
                writes = []
                for L in range(64):
                    q = 16 * L + k
                    first, low = quad_words_at(b, q)
                    writes += [(L, o[L], first), (L, o[L] + 1, low)]
                    o[L] += width[q]
                for L, a, v in sorted(writes, key=lambda w: w[0], reverse=(order == "high")):
                    stage[a] = v
            for L in range(64):
                pos = [16 * L + k for k in range(8) if lead[16 * L + k]]
                if not pos or pos[0] >= 16 * L + 4:
                    continue
                p1 = pos[0]
                stage[base[L]] = quad_words_at(b, p1)[0]
                if b[p1] >= 0xF0:
                    stage[base[L] + 1] = quad_words_at(b, p1)[1]
                elif len(pos) > 1:
                    stage[base[L] + 1] = quad_words_at(b, pos[1])[0]
            ref = []
            i = 0
            for cp in cps:
                if i >= 1024:
                    break
                ref += list(np.frombuffer(chr(cp).encode("utf-16-le"), dtype="<u2"))
                i += len(chr(cp).encode("utf-8"))
            total = sum(lw)
            assert [stage.get(s) for s in range(total)] == [int(x) for x in ref[:total]], (trial, order)


def test_surrogate_pair_bytes_split_by_word():
    """The UTF-16 -> UTF-8 kernels encode a surrogate pair word by word: the
    high word alone gives the first two bytes (through v >> 12 =
    0x10 + ((hi >> 2) & 0xFF)) and the low word the last two, with two bits
    (hi & 3) taken from the word before it.  Every pair, against Python's
    own encoder."""
    hi = np.repeat(np.arange(0xD800, 0xDC00, dtype=np.uint32), 1024)
    lo = np.tile(np.arange(0xDC00, 0xE000, dtype=np.uint32), 1024)
    v12 = ((hi >> 2) & 0xFF) + 0x10
    got = np.stack([(v12 >> 6) | 0xF0, (v12 & 0x3F) | 0x80,
                    ((hi & 3) << 4) | ((lo >> 6) & 0xF) | 0x80, (lo & 0x3F) | 0x80], axis=1).astype(np.uint8)
    cp = 0x10000 + ((hi & 0x3FF) << 10 | (lo & 0x3FF))
    text = "".join(map(chr, cp.tolist()))
    want = np.frombuffer(text.encode("utf-8"), dtype=np.uint8).reshape(-1, 4)
    assert np.array_equal(got, want)


def _alignbyte(a, b, k):
    """v_alignbyte_b32: bytes k..k+3 of the 8-byte value (a << 32 | b)."""
    return ((a << 32 | b) >> (8 * k)) & 0xFFFFFFFF


@pytest.mark.parametrize("rows", [2, 4])
def test_ascii_narrow_store_blocks(rows):
    """Model of the UTF-16 -> UTF-8 all-ASCII direct store: for every
    alignment of the wave's first output byte, the aligned 8-byte blocks of
    lane-rows 1.. plus the head and tail byte stores write exactly the
    wave's 512 * rows bytes, each once, with the right values."""
    n = 512 * rows
    rng = np.random.default_rng(rows)
    wave = rng.integers(0, 128, size=n, dtype=np.uint64)
    for base in range(8, 24):
        s8 = base & 7
        o = 8 - s8
        mem = {}
        lane_rows = [(int(sum(int(wave[8 * q + i]) << (8 * i) for i in range(4))),
                      int(sum(int(wave[8 * q + 4 + i]) << (8 * i) for i in range(4)))) for q in range(n // 8)]
        for q, (lo, hi) in enumerate(lane_rows):
            def put(addr, byte):
                assert addr not in mem, (base, q, addr)
                mem[addr] = byte
            if s8 == 0:
                for i in range(8):
                    put(base + 8 * q + i, ((lo | hi << 32) >> (8 * i)) & 0xFF)
                continue
            plo, phi = lane_rows[q - 1] if q > 0 else (0, 0)
            if o < 4:
                a, b = _alignbyte(phi, plo, o), _alignbyte(lo, phi, o)
            else:
                a, b = _alignbyte(lo, phi, o - 4), _alignbyte(hi, lo, o - 4)
            if q > 0:
                blk = a | b << 32
                for i in range(8):
                    put(base - s8 + 8 * q + i, (blk >> (8 * i)) & 0xFF)
            else:
                for i in range(o):
                    put(base + i, ((lo | hi << 32) >> (8 * i)) & 0xFF)
            if q == n // 8 - 1:
                for i in range(o, 8):
                    put(base + 8 * q + i, ((lo | hi << 32) >> (8 * i)) & 0xFF)
        assert sorted(mem) == list(range(base, base + n)), base
        assert all(mem[base + i] == int(wave[i]) for i in range(n)), base


# --------------------------------------------------------------------------
# 8. Weighted byte sums (v_dot4_u32_u8) decode a window.  For the window
#    w = b0 | b1 << 8 | b2 << 16 | b3 << 24 the windows decoder forms
#      v2 = 64 b0 + b1 - 0x3080, v3 = 64 v2 + b2 - 0x20080,
#      v4 = 4096 v2 + 64 b2 + b3 - 0xC02080          (all modulo 2^32)
#    and for a leading byte >= F0 the surrogates 0xD7C0 + (v4 >> 10) and
#    0xDC00 | (v4 & 0x3FF); a marked copy (first byte xor 0x70) must give the
#    same low surrogate.  Its value flags are: C0/C1; a three-byte lead whose
#    v3 >> 11 is 0 or 27 (below U+0800, or U+D800..DFFF); a lead >= F0 whose
#    v4 - 0x10000 exceeds 0xFFFFF.
# --------------------------------------------------------------------------

M32 = (1 << 32) - 1


def _dot4(w, weights, addend):
    s = np.zeros_like(w)
    for k in range(4):
        s = s + ((w >> (8 * k)) & 0xFF) * ((weights >> (8 * k)) & 0xFF)
    return (s + addend) & M32


def _decode_model(w):
    """(word, bad) of the kAny windows decoder for uint64 windows w."""
    b0 = w & 0xFF
    v2 = _dot4(w, 0x00000140, (-0x3080) & M32)
    v3 = _dot4(w, 0x00010000, ((v2 << 6) - 0x20080) & M32)
    v4 = _dot4(w, 0x01400000, ((v2 << 12) - 0xC02080) & M32)
    l3, l4 = b0 >= 0xE0, b0 >= 0xF0
    b3 = ((0x08000001 >> ((v3 >> 11) & 31)) & 1) == 1
    bad = ((w & 0xFE) == 0xC0) | (l3 & ~l4 & b3) | (l4 & (((v4 - 0x10000) & M32) > 0xFFFFF))
    hi, lo = (0xD7C0 + (v4 >> 10)) & 0xFFFF, 0xDC00 | (v4 & 0x3FF)
    u = np.where(l3, v3, np.where(b0 >= 0xC0, v2, b0)) & 0xFFFF
    word = np.where(l4, hi, np.where((b0 & 0xC0) == 0x80, lo, u))
    return word, bad


def test_weighted_sums_decode_every_scalar_value():
    """Every scalar value: the window of its UTF-8 form decodes to its first
    UTF-16 word (Python's encoders), the marked copy of a four-byte form to
    its low surrogate, and no value flag is raised."""
    cps = [c for c in range(0x110000) if not 0xD800 <= c <= 0xDFFF]
    text = "".join(map(chr, cps))
    u8 = text.encode("utf-8")
    lens = np.array([1 if c < 0x80 else 2 if c < 0x800 else 3 if c < 0x10000 else 4 for c in cps])
    starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
    buf = np.frombuffer(u8 + b"\0\0\0", dtype=np.uint8).astype(np.uint64)
    w = buf[starts] | buf[starts + 1] << 8 | buf[starts + 2] << 16 | buf[starts + 3] << 24
    w = np.where(lens == 1, w & 0xFF, np.where(lens == 2, w & 0xFFFF, np.where(lens == 3, w & 0xFFFFFF, w)))
    word, bad = _decode_model(w)
    u16 = np.frombuffer(text.encode("utf-16-le"), dtype="<u2").astype(np.uint64)
    first = np.concatenate([[0], np.cumsum(np.where(lens == 4, 2, 1))[:-1]])
    assert not bad.any()
    assert np.array_equal(word, u16[first])
    four = lens == 4
    lo_word, lo_bad = _decode_model(w[four] ^ 0x70)
    assert np.array_equal(lo_word, u16[first[four] + 1])


@pytest.mark.parametrize("lead", range(0xC0, 0x100))
def test_weighted_sums_value_flags_match_the_rules(orc, lead):
    """Every window of one leading byte followed by the continuation bytes it
    announces (all 64^(L-1) of them, L = 2, 3, 4; L = 4 for F8..FF too): the
    value flag is raised exactly when the oracle rejects the sequence (its
    structure being complete, only rules 1, 4, 5, 6 can fail)."""
    L = 2 if lead < 0xE0 else 3 if lead < 0xF0 else 4
    conts = np.arange(0x80, 0xC0, dtype=np.uint64)
    grids = np.meshgrid(*([conts] * (L - 1)), indexing="ij")
    w = np.full(grids[0].size, lead, dtype=np.uint64)
    for k, g in enumerate(grids):
        w |= g.reshape(-1) << (8 * (k + 1))
    _, bad = _decode_model(w)
    data = np.stack([(w >> (8 * k)) & 0xFF for k in range(L)], axis=1).astype(np.uint8).reshape(-1)
    st, _ = orc.validate_utf8_batch(data, np.arange(0, data.size + 1, L, dtype=np.int64))
    assert np.array_equal(bad, st != O.OK)


# ---------------------------------------------------------------------------
# Batched calls: the owner of every wave span without a search.  The span
# owner is defined as the largest i with offsets[i] <= p for the span's first
# position p (clamped to [0, n - 1]), i.e. a binary search; the prep kernel
# instead lets string i write itself into every span w whose first position
# it holds: w from ceil((a + head) / span) (from 0 when a = 0) to
# ceil((b + head) / span) - 1 (to the last span when b = n).  For offsets
# that partition [0, n] the two agree on every span.
# ---------------------------------------------------------------------------
def _owner_by_search(offsets, p):
    lo, hi = 0, len(offsets) - 1
    while hi > lo + 1:
        mid = (lo + hi) // 2
        if offsets[mid] <= p:
            lo = mid
        else:
            hi = mid
    return lo


def _owners_by_strings(offsets, head, span, nspans):
    n = offsets[-1]
    own = [None] * (nspans + 1)
    for i in range(len(offsets) - 1):
        a, b = offsets[i], offsets[i + 1]
        if a == b:
            continue
        wlo = 0 if a == 0 else (a + head + span - 1) // span
        whi = nspans if b == n else (b + head + span - 1) // span - 1
        for w in range(wlo, whi + 1):
            own[w] = i
    return own


def test_span_owners_without_search():
    rng = np.random.default_rng(17)
    for _ in range(4000):
        k = int(rng.integers(1, 40))
        lens = rng.integers(0, 300, size=k) * (rng.random(k) < 0.8)
        if lens.sum() == 0:
            lens[int(rng.integers(0, k))] = int(rng.integers(1, 50))
        offsets = [0] + np.cumsum(lens).astype(int).tolist()
        n = offsets[-1]
        head = int(rng.integers(0, 16))
        span = int(rng.choice([16, 64, 128, 2048]))
        nspans = 4 * ((head + n + 4 * span - 1) // (4 * span))
        want = []
        for w in range(nspans + 1):
            p = min(max(w * span - head, 0), n - 1)
            want.append(_owner_by_search(offsets, p))
        assert _owners_by_strings(offsets, head, span, nspans) == want, (offsets, head, span)


def test_edge_width_correction():
    """Waves at the ends of the input: the bytes outside [head, end) are
    zeroed before the survey, so counting a chunk's output words over all 16
    positions (one per non-continuation byte, one more per byte >= F0) and
    then taking off the positions outside the input, in closed form
    (16 - |[q0, q0 + 16) & [head, end)|), gives the count over the chunk's
    own positions: a zero byte is neither a continuation nor >= F0."""
    rng = np.random.default_rng(21)
    for _ in range(4000):
        head = int(rng.integers(0, 48))
        end = head + int(rng.integers(0, 96))
        q0 = 16 * int(rng.integers(-2, 10))
        raw = rng.integers(0, 256, size=16)
        inside = [head <= q0 + i < end for i in range(16)]
        b = [int(x) if ins else 0 for x, ins in zip(raw, inside)]
        own = sum((1 + (x >= 0xF0)) for x, ins in zip(b, inside) if ins and (x & 0xC0) != 0x80)
        every = sum((1 + (x >= 0xF0)) for x in b if (x & 0xC0) != 0x80)
        a, z = max(q0, head), min(q0 + 16, end)
        outside = 16 - (z - a if z > a else 0)
        assert outside == sum(not ins for ins in inside)
        assert every - outside == own


# 6. Row write-out with carried blocks.  A wave stages each row's output
#    [g0, g1) by 16-byte blocks of global memory (byte g at stage byte
#    g - (g0 & ~15)) and stores it: lane i takes blocks i, i + 64, ... up to
#    the row's last whole block; the row's unfinished last block is carried
#    to the next row, whose block 0 it completes (in registers); a block
#    that begins before the wave's first byte `wstart` is stored in part
#    with aligned stores of 1..8 bytes (never below the unit size); after
#    a row cut short (the next row starts further on) and at the wave's end
#    the carried block is stored in part.  Every byte of every row must be
#    written once with its value; the gap after a row cut short (which only
#    happens past an error, where the output is unspecified) may be written
#    once with any value; nothing else is written.

def store_part(mem, c, a, b, block, unit):
    for sz in (1, 2, 4, 8):   # up to the first 16-byte aligned chunk
        if sz >= unit and (a & sz) and a + sz <= b:
            for j in range(sz):
                mem.append((a + j, block[a - c + j], sz, a))
            a += sz
    for sz in (8, 4, 2, 1):   # the rest, largest first
        if sz >= unit and a + sz <= b:
            for j in range(sz):
                mem.append((a + j, block[a - c + j], sz, a))
            a += sz
    assert a == b, (c, a, b)


def write_row_model(mem, g0, g1, wstart, stage, carry, merge, unit):
    c0 = g0 & ~15
    lo = max(c0, wstart)
    hi = g1 & ~15
    k = g0 & 15
    merge = merge and k != 0
    nb = (hi - c0) >> 4
    part0 = c0 < lo
    for b in range(nb):
        block = list(stage[16 * b:16 * b + 16])
        if b == 0 and merge:
            block[:k] = carry[:k]
        if b == 0 and part0:
            store_part(mem, c0, lo, c0 + 16, block, unit)
        else:
            mem.extend((c0 + 16 * b + j, block[j], 16, c0 + 16 * b) for j in range(16))
    if g1 & 15:
        blk = list(stage[hi - c0:hi - c0 + 16])
        if merge and nb == 0:
            blk[:k] = carry[:k]
        carry = blk
    return carry


@pytest.mark.parametrize("unit", [1, 2])
def test_row_write_out_with_carry(unit):
    rng = np.random.default_rng(31 + unit)
    for trial in range(3000):
        wstart = 4096 + unit * int(rng.integers(0, 64 // unit))
        rows, u, gap = [], wstart, set()
        for _ in range(int(rng.integers(1, 6))):
            if rng.random() < 0.15:   # a row cut short before: the next one starts further on
                g = unit * int(rng.integers(1, 40))
                gap.update(range(u, u + g))
                u += g
            n = unit * int(rng.choice([0, 1, 2, 3, 7, 8, 9, 15, 16, 17, 100, 1000, 1032]))
            rows.append((u, u + n))
            u += n
        want = {}
        mem, carry, wlo, gend = [], [0] * 16, wstart, wstart
        for g0, g1 in rows:
            value = lambda a: (a * 131 + trial) & 0xFF
            stage = [int(x) for x in rng.integers(0, 256, size=16 * ((g1 - (g0 & ~15)) // 16 + 2))]
            for a in range(g0, g1):
                stage[a - (g0 & ~15)] = value(a)
                want[a] = value(a)
            if g0 < g1 and gend != g0:
                if gend & 15:
                    c = gend & ~15
                    store_part(mem, c, max(c, wlo), gend, carry, unit)
                wlo = gend
            if g0 < g1:
                carry = write_row_model(mem, g0, g1, wlo, stage, carry, gend == g0 and gend > wlo, unit)
                gend = g1
        if gend & 15:
            c = gend & ~15
            store_part(mem, c, max(c, wlo), gend, carry, unit)
        got = {}
        for a, v, sz, base in mem:
            assert base % sz == 0 and sz >= unit, (trial, a, sz)
            assert a not in got, (trial, a)    # each byte once
            got[a] = v
        assert {a: v for a, v in got.items() if a not in gap} == want, trial
        assert all(a < gend for a in got if a in gap), trial
