"""Seeded synthetic text generators for UTF-8 / UTF-16LE workloads.

The paper measures on multilingual lipsum files that are not available here;
these generators stand in for them with i.i.d. code points drawn per
character class.  This module holds no transcoding arithmetic of its own:
code points are drawn with numpy (PCG64) and turned into bytes by CPython's
strict codecs (``str.encode``).  Invalid variants are built by splicing fixed
invalid byte patterns (test data) between encoded runs of valid characters,
so the generator knows exactly where each error starts.

Every buffer is a pure function of (mix, size, seed, error rate).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Character classes and mixes
# --------------------------------------------------------------------------

# Printable ASCII U+0020..U+007E.
ASCII_PRINTABLE = np.arange(0x20, 0x7F, dtype=np.uint32)
# ASCII spaces and punctuation: U+0020..002F, 003A..0040, 005B..0060, 007B..007E.
ASCII_PUNCT = np.concatenate([
    np.arange(0x20, 0x30), np.arange(0x3A, 0x41), np.arange(0x5B, 0x61), np.arange(0x7B, 0x7F),
]).astype(np.uint32)


def _span(lo: int, hi: int) -> np.ndarray:
    return np.arange(lo, hi + 1, dtype=np.uint32)


# U+0800..U+FFFF without the surrogate block U+D800..U+DFFF.
_BMP3 = np.concatenate([_span(0x800, 0xD7FF), _span(0xE000, 0xFFFF)])

# mix name -> list of (weight, values drawn uniformly)
MIXES: Dict[str, List[Tuple[float, np.ndarray]]] = {
    # Single-buffer 1 MiB case: half printable ASCII, then 2-, 3- and 4-byte ranges.
    "mix1m": [(0.50, ASCII_PRINTABLE), (0.25, _span(0x80, 0x7FF)),
              (0.20, _BMP3), (0.05, _span(0x10000, 0x10FFFF))],
    "ascii": [(1.0, ASCII_PRINTABLE)],
    "latin": [(0.90, ASCII_PRINTABLE), (0.10, _span(0xC0, 0x17F))],
    "cyrillic": [(0.15, ASCII_PUNCT), (0.85, _span(0x400, 0x4FF))],
    "cjk": [(0.10, ASCII_PRINTABLE), (0.90, _span(0x4E00, 0x9FFF))],
    "emoji": [(0.70, ASCII_PRINTABLE), (0.30, _span(0x1F300, 0x1FAFF))],
}
SCRIPT_MIXES = ("ascii", "latin", "cyrillic", "cjk", "emoji")

# Seeds (one stream per purpose).
SEED_MIX1M = 1
SEED_UTF8 = {m: 100 + k for k, m in enumerate(SCRIPT_MIXES)}
SEED_UTF8_INVALID = {m: 200 + k for k, m in enumerate(SCRIPT_MIXES)}
SEED_UTF16 = {m: 300 + k for k, m in enumerate(SCRIPT_MIXES)}
SEED_UTF16_INVALID = {m: 400 + k for k, m in enumerate(SCRIPT_MIXES)}
SEED_BATCH = 500
SEED_SERVE = 600

# Invalid UTF-8 patterns.  Each entry: (name, list of byte ranges).  The
# error of every pattern sits on its first byte when it follows a complete
# character and precedes a character start.
UTF8_BAD_PATTERNS: List[Tuple[str, List[Tuple[int, int]]]] = [
    ("overlong2", [(0xC0, 0xC1), (0x80, 0xBF)]),
    ("overlong3", [(0xE0, 0xE0), (0x80, 0x9F), (0x80, 0xBF)]),
    ("overlong4", [(0xF0, 0xF0), (0x80, 0x8F), (0x80, 0xBF), (0x80, 0xBF)]),
    ("surrogate", [(0xED, 0xED), (0xA0, 0xBF), (0x80, 0xBF)]),
    ("too_large_f4", [(0xF4, 0xF4), (0x90, 0xBF), (0x80, 0xBF), (0x80, 0xBF)]),
    ("too_large_f5", [(0xF5, 0xF7), (0x80, 0xBF), (0x80, 0xBF), (0x80, 0xBF)]),
    ("stray_continuation", [(0x80, 0xBF)]),
    ("truncated2", [(0xC2, 0xDF)]),
    ("truncated3", [(0xE1, 0xEC), (0x80, 0xBF)]),
    ("truncated4", [(0xF1, 0xF3), (0x80, 0xBF), (0x80, 0xBF)]),
    ("header_bits", [(0xF8, 0xFF)]),
]
# Unpaired surrogates for UTF-16.
UTF16_BAD_PATTERNS: List[Tuple[str, Tuple[int, int]]] = [
    ("unpaired_high", (0xD800, 0xDBFF)),
    ("unpaired_low", (0xDC00, 0xDFFF)),
]

CHUNK_CHARS = 1 << 22


# --------------------------------------------------------------------------
# Drawing code points
# --------------------------------------------------------------------------

def draw_codepoints(rng: np.random.Generator, mix: str, count: int) -> np.ndarray:
    """``count`` i.i.d. code points of ``mix`` as uint32.

    One uniform number u per character picks both the class (the interval
    of the cumulative weights u falls in) and the value inside the class
    (u's position inside that interval, scaled to the class size)."""
    classes = MIXES[mix]
    if len(classes) == 1:
        vals = classes[0][1]
        return vals[rng.integers(0, vals.size, size=count)]
    w = np.array([c[0] for c in classes], dtype=np.float64)
    w /= w.sum()
    hi = np.cumsum(w)
    hi[-1] = 1.0
    lo = hi - w
    sizes = np.array([c[1].size for c in classes], dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    table = np.concatenate([c[1] for c in classes])
    u = rng.random(count)
    cls = np.minimum(np.searchsorted(hi, u, side="right"), len(classes) - 1)
    idx = ((u - lo[cls]) / w[cls] * sizes[cls]).astype(np.int64)
    idx = np.clip(idx, 0, sizes[cls] - 1)
    return table[starts[cls] + idx]


def _to_str(cps: np.ndarray) -> str:
    return cps.astype("<u4").tobytes().decode("utf-32-le")


def _encode(cps: np.ndarray, enc: str) -> bytes:
    return _to_str(cps).encode(enc)


# --------------------------------------------------------------------------
# Invalid patterns
# --------------------------------------------------------------------------

def _utf8_bad(rng: np.random.Generator) -> Tuple[str, bytes]:
    name, ranges = UTF8_BAD_PATTERNS[int(rng.integers(0, len(UTF8_BAD_PATTERNS)))]
    return name, bytes(int(rng.integers(lo, hi + 1)) for lo, hi in ranges)


def _utf16_bad(rng: np.random.Generator) -> Tuple[str, bytes]:
    name, (lo, hi) = UTF16_BAD_PATTERNS[int(rng.integers(0, len(UTF16_BAD_PATTERNS)))]
    return name, int(rng.integers(lo, hi + 1)).to_bytes(2, "little")


# --------------------------------------------------------------------------
# Fixed-size buffers
# --------------------------------------------------------------------------

@dataclass
class TextBuffer:
    """A generated buffer and what the generator knows about it."""
    mix: str
    encoding: str                # "utf-8" or "utf-16-le"
    data: np.ndarray             # uint8 (UTF-8) or uint16 (UTF-16LE)
    pad: int                     # padding units (U+0020) at the end
    errors: List[Tuple[int, str]] = field(default_factory=list)  # (unit offset, pattern), ascending

    @property
    def first_error(self) -> Optional[int]:
        return self.errors[0][0] if self.errors else None


_PER_CHAR = {"utf-8": {"mix1m": 2.0, "ascii": 1.0, "latin": 1.1, "cyrillic": 1.85, "cjk": 2.8, "emoji": 1.9},
             "utf-16-le": {"mix1m": 2.1, "ascii": 2.0, "latin": 2.0, "cyrillic": 2.0, "cjk": 2.0, "emoji": 2.6}}


def _chunk_pieces(mix: str, encoding: str, seq: np.random.SeedSequence, nchars: int,
                  bad: List[Tuple[int, str, bytes]]) -> List[Tuple[Optional[str], bytes]]:
    """Draw ``nchars`` characters; replace the characters at the (relative)
    indices in ``bad`` by their patterns.  Returns the ordered pieces:
    ``(None, encoded run)`` or ``(pattern name, pattern bytes)``."""
    rng = np.random.Generator(np.random.PCG64(seq))
    cps = draw_codepoints(rng, mix, nchars)
    pieces: List[Tuple[Optional[str], bytes]] = []
    cursor = 0
    for rel, name, pat in bad:
        pieces.append((None, _encode(cps[cursor:rel], encoding)))
        pieces.append((name, pat))
        cursor = rel + 1
    pieces.append((None, _encode(cps[cursor:], encoding)))
    return pieces


def make_buffer(mix: str, size_bytes: int, seed: int, encoding: str = "utf-8",
                error_rate: float = 0.0, error_seed: Optional[int] = None,
                workers: Optional[int] = None, executor=None) -> TextBuffer:
    """A buffer of exactly ``size_bytes`` bytes of ``mix`` text.

    Characters are drawn chunk by chunk (``CHUNK_CHARS`` per chunk, chunk j
    seeded by child j of ``SeedSequence(seed)``) and appended until the next
    one would not fit; the rest is padded with U+0020.  With
    ``error_rate > 0``, ``round(units * error_rate)`` characters (at least one)
    at seeded character indices, kept at least three characters apart, are
    replaced by invalid patterns; ``errors`` lists the unit offset of each
    pattern that made it into the buffer.

    ``executor`` (e.g. a process pool) draws and encodes chunks in
    parallel; by default a thread pool is used.  The result does not depend
    on it.
    """
    unit = 1 if encoding == "utf-8" else 2
    assert size_bytes % unit == 0 and size_bytes >= 0
    units_total = size_bytes // unit
    est_chars = int(size_bytes / _PER_CHAR[encoding][mix] * 1.02) + 64
    nchunks = max(1, math.ceil(est_chars / CHUNK_CHARS)) + 8
    seqs = np.random.SeedSequence(seed).spawn(nchunks)

    # Injected characters (global character index -> pattern), drawn up front.
    bad_by_chunk: Dict[int, List[Tuple[int, str, bytes]]] = {}
    if error_rate > 0 and units_total > 0:
        nerr = max(1, int(round(units_total * error_rate)))
        erng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
            error_seed if error_seed is not None else seed + 7919)))
        span = max(int(est_chars * 0.95), nerr * 4)
        cand = np.sort(erng.choice(span, size=nerr, replace=False))
        keep = [int(cand[0])]
        for c in cand[1:]:
            if int(c) > keep[-1] + 2:
                keep.append(int(c))
        for c in keep:
            name, pat = _utf8_bad(erng) if encoding == "utf-8" else _utf16_bad(erng)
            bad_by_chunk.setdefault(c // CHUNK_CHARS, []).append((c % CHUNK_CHARS, name, pat))

    out = np.empty(size_bytes, dtype=np.uint8)
    filled = 0
    errors: List[Tuple[int, str]] = []
    workers = workers or min(16, os.cpu_count() or 1)

    def place(pieces) -> bool:
        """Copy pieces in order; on overflow cut the run at a character
        boundary (CPython drops the incomplete tail) and report False."""
        nonlocal filled
        for name, blob in pieces:
            room = size_bytes - filled
            if len(blob) > room:
                if name is None:
                    cut = room - room % unit
                    head = blob[:cut].decode(encoding, errors="ignore").encode(encoding)
                    out[filled:filled + len(head)] = np.frombuffer(head, dtype=np.uint8)
                    filled += len(head)
                return False
            if name is not None:
                errors.append((filled // unit, name))
            out[filled:filled + len(blob)] = np.frombuffer(blob, dtype=np.uint8)
            filled += len(blob)
        return True

    own = executor is None
    ex = ThreadPoolExecutor(max_workers=workers) if own else executor
    try:
        j = 0
        full = True
        while full:
            if j >= nchunks:
                raise RuntimeError("generator ran out of chunks")
            batch = list(range(j, min(j + workers, nchunks)))
            futs = [ex.submit(_chunk_pieces, mix, encoding, seqs[c], CHUNK_CHARS, bad_by_chunk.get(c, []))
                    for c in batch]
            for f in futs:
                if full and not place(f.result()):
                    full = False
            j = batch[-1] + 1
    finally:
        if own:
            ex.shutdown()

    pad = size_bytes - filled
    out[filled:] = 0x20
    if unit == 2:
        out[filled + 1::2] = 0x00
        data = out.view("<u2")
    else:
        data = out
    return TextBuffer(mix=mix, encoding=encoding, data=data, pad=pad // unit, errors=errors)


# --------------------------------------------------------------------------
# Many strings (batched workload)
# --------------------------------------------------------------------------

@dataclass
class StringBatch:
    data: np.ndarray            # concatenated uint8 (UTF-8) or uint16 (UTF-16LE)
    offsets: np.ndarray         # int64[k+1], in units
    mixes: List[str]
    errors: Dict[int, int]      # string index -> first-error offset inside the string


def lognormal_lengths(rng: np.random.Generator, k: int, median: float, sigma: float,
                      lo: int, hi: int) -> np.ndarray:
    x = rng.lognormal(mean=math.log(median), sigma=sigma, size=k)
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def _one_string(rng: np.random.Generator, mix: str, nbytes: int, encoding: str,
                inject: bool) -> Tuple[bytes, Optional[int]]:
    unit = 1 if encoding == "utf-8" else 2
    nbytes -= nbytes % unit
    per_char = 1.0 if mix == "ascii" else 1.5
    count = int(nbytes / per_char) + 8
    cps = draw_codepoints(rng, mix, count)
    s = _to_str(cps)
    enc = s.encode(encoding)
    if len(enc) > nbytes:
        enc = enc[:nbytes].decode(encoding, errors="ignore").encode(encoding)
    err = None
    if inject:
        # replace a character at a seeded index
        t = enc.decode(encoding)
        if len(t) >= 1:
            ci = int(rng.integers(0, len(t)))
            _, pat = _utf8_bad(rng) if encoding == "utf-8" else _utf16_bad(rng)
            head = t[:ci].encode(encoding)
            tail = t[ci + 1:].encode(encoding)
            enc = head + pat + tail
            if len(enc) > nbytes:
                enc = enc[:nbytes]
                if len(head) + len(pat) > nbytes:
                    enc = head  # pattern would not fit: no error
                else:
                    # cut the tail at a character boundary
                    room = nbytes - len(head) - len(pat)
                    enc = head + pat + tail[:room].decode(encoding, errors="ignore").encode(encoding)
            if len(enc) >= len(head) + len(pat) and enc[len(head):len(head) + len(pat)] == pat:
                err = len(head) // unit
    pad = nbytes - len(enc)
    enc += (b" " if unit == 1 else b" \x00") * (pad // unit)
    return enc, err


def make_batch(k: int = 100_000, seed: int = SEED_BATCH, encoding: str = "utf-8",
               median: float = 256, sigma: float = 1.5, lo: int = 16, hi: int = 1 << 20,
               error_fraction: float = 0.01, mixes: Sequence[str] = SCRIPT_MIXES) -> StringBatch:
    """``k`` independent strings with log-normal byte lengths, one mix each
    (chosen uniformly), ``error_fraction`` of them with one injected error."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    lengths = lognormal_lengths(rng, k, median, sigma, lo, hi)
    mix_idx = rng.integers(0, len(mixes), size=k)
    nerr = int(round(k * error_fraction))
    bad = set(int(x) for x in rng.choice(k, size=nerr, replace=False)) if nerr else set()
    seqs = np.random.SeedSequence(seed + 1).spawn(k)
    parts: List[bytes] = []
    errors: Dict[int, int] = {}
    for i in range(k):
        r = np.random.Generator(np.random.PCG64(seqs[i]))
        enc, e = _one_string(r, mixes[int(mix_idx[i])], int(lengths[i]), encoding, i in bad)
        parts.append(enc)
        if e is not None:
            errors[i] = e
    unit = 1 if encoding == "utf-8" else 2
    blob = b"".join(parts)
    offsets = np.zeros(k + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(p) // unit for p in parts])
    data = np.frombuffer(blob, dtype=np.uint8 if unit == 1 else "<u2").copy()
    return StringBatch(data=data, offsets=offsets, mixes=[mixes[int(m)] for m in mix_idx], errors=errors)


def random_text(rng: np.random.Generator, mix: str, nchars: int, encoding: str = "utf-8") -> np.ndarray:
    """Small helper: ``nchars`` characters of ``mix`` encoded as a numpy array."""
    b = _encode(draw_codepoints(rng, mix, nchars), encoding)
    return np.frombuffer(b, dtype=np.uint8 if encoding == "utf-8" else "<u2").copy()


# --------------------------------------------------------------------------
# Serving: an open-loop request stream
# --------------------------------------------------------------------------

@dataclass
class RequestSet:
    """Requests in arrival order.  ``kind`` 0 is UTF-8 -> UTF-16LE, 1 the
    reverse.  The payloads of each kind lie back to back in ``data8`` /
    ``data16`` in arrival order: request ``ids8[j]`` is
    ``data8[off8[j]:off8[j+1]]`` (bytes), request ``ids16[j]`` is
    ``data16[off16[j]:off16[j+1]]`` (16-bit units)."""
    arrival: np.ndarray          # seconds after the start, ascending
    kind: np.ndarray             # int8
    size: np.ndarray             # payload bytes
    mixes: List[str]
    invalid: np.ndarray          # bool: one byte or unit was replaced
    ids8: np.ndarray
    off8: np.ndarray
    data8: np.ndarray
    ids16: np.ndarray
    off16: np.ndarray
    data16: np.ndarray


def _char_start8(pool: np.ndarray, i: int) -> int:
    while i < pool.size and (pool[i] & 0xC0) == 0x80:
        i += 1
    return i


def _char_start16(pool: np.ndarray, i: int) -> int:
    return i + 1 if i < pool.size and 0xDC00 <= pool[i] <= 0xDFFF else i


def make_requests(n: int, rate: float = 50_000.0, seed: int = SEED_SERVE, median: float = 32768,
                  sigma: float = math.log(2 ** 18) / 6, lo: int = 64, hi: int = 16 << 20,
                  invalid_fraction: float = 0.005, pool_bytes: int = 32 << 20,
                  mixes: Sequence[str] = SCRIPT_MIXES, executor=None) -> RequestSet:
    """``n`` requests with Poisson arrivals at ``rate`` per second, log-normal
    payload sizes (``median``, ``sigma``, clipped to [lo, hi]), direction
    50/50, mix uniform, ``invalid_fraction`` with one replaced byte (0xFF) or
    unit (a lone low surrogate).  Payloads are slices of one generated pool
    per mix and encoding, cut at character boundaries."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=n))
    kind = rng.integers(0, 2, size=n).astype(np.int8)
    size = lognormal_lengths(rng, n, median, sigma, lo, min(hi, pool_bytes // 2))
    mix_idx = rng.integers(0, len(mixes), size=n)
    invalid = rng.random(n) < invalid_fraction
    pools8 = {m: make_buffer(m, pool_bytes, seed + 10 + k, executor=executor).data for k, m in enumerate(mixes)}
    pools16 = {m: make_buffer(m, pool_bytes, seed + 20 + k, encoding="utf-16-le", executor=executor).data
               for k, m in enumerate(mixes)}
    parts8, parts16, ids8, ids16 = [], [], [], []
    for i in range(n):
        mix = mixes[int(mix_idx[i])]
        if kind[i] == 0:
            pool = pools8[mix]
            a = _char_start8(pool, int(rng.integers(0, pool.size - size[i])))
            b = _char_start8(pool, a + int(size[i]))
            p = pool[a:b].copy()
            if invalid[i] and p.size:
                p[int(rng.integers(0, p.size))] = 0xFF
            parts8.append(p)
            ids8.append(i)
        else:
            pool = pools16[mix]
            units = int(size[i]) // 2
            a = _char_start16(pool, int(rng.integers(0, pool.size - units)))
            b = _char_start16(pool, a + units)
            p = pool[a:b].copy()
            if invalid[i] and p.size:
                p[int(rng.integers(0, p.size))] = 0xDC00
            parts16.append(p)
            ids16.append(i)
        size[i] = p.nbytes
    off8 = np.zeros(len(parts8) + 1, dtype=np.int64)
    off8[1:] = np.cumsum([p.size for p in parts8])
    off16 = np.zeros(len(parts16) + 1, dtype=np.int64)
    off16[1:] = np.cumsum([p.size for p in parts16])
    data8 = np.concatenate(parts8) if parts8 else np.zeros(0, np.uint8)
    data16 = np.concatenate(parts16) if parts16 else np.zeros(0, np.uint16)
    return RequestSet(arrival=arrival, kind=kind, size=size, mixes=[mixes[int(m)] for m in mix_idx],
                      invalid=invalid, ids8=np.array(ids8, dtype=np.int64), off8=off8, data8=data8,
                      ids16=np.array(ids16, dtype=np.int64), off16=off16, data16=data16)
