"""GPU parity of every compiled tile geometry in both scan schedules, and
of the tuner's tables.

Each (geometry, schedule) pair is forced for every operation and size
class, and the single-buffer and batched calls are checked against the CPU
oracle, bit for bit, at sizes and positions placed on that geometry's own
row, wave and tile boundaries (ragged tails, straddling characters and
errors, random bytes, stage overflow).  The rest of the suite runs the
shipped tables (8 KiB tiles up to 4 MiB, the 8 x 4 build above, for most
calls; block order everywhere).  Then a short tuning run must produce tables
that name compiled geometries and known schedules, install them, survive a
JSON round trip, and leave every result unchanged.
"""
import numpy as np
import pytest
import torch

import oracle as O
from tests.test_gpu_batch import check_batch, check_batch16, pack
from tests.test_gpu_parity import _filler, _utf8_patterns, check_utf8, check_utf16
from workloads import random_text
from workloads.mixes import SEED_BATCH, make_batch, make_buffer

pytestmark = pytest.mark.gpu

try:
    import paper_2111_08692_amd as _G
    _NGEOM = len(_G.geometries())
except Exception:   # library not built: the tests below fail in the fixture
    _NGEOM = 2


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2111_08692_amd as G
    G.load()
    return G


def _force(G, g, s=-1):
    for op in range(G.OP_COUNT):
        for c in range(G.SIZE_CLASSES):
            assert G.set_geometry(op, c, g) == G.OK
            assert G.set_schedule(op, c, s) == G.OK


_PAIRS = [(g, s) for s in (0, 1) for g in range(_NGEOM)]


@pytest.fixture(params=_PAIRS, ids=lambda p: f"geometry{p[0]}-{('block', 'ticket')[p[1]]}")
def geom(G, request):
    g, s = request.param
    waves, rows, tile = G.geometries()[g]
    _force(G, g, s)
    assert all(G.get_geometry(op, c) == g and G.get_schedule(op, c) == s
               for op in range(G.OP_COUNT) for c in (0, 17, 40))
    yield {"index": g, "schedule": s, "waves": waves, "rows": rows, "tile": tile, "wave": rows * 1024}
    _force(G, -1)


MIXES = ("mix1m", "ascii", "latin", "cjk", "emoji")


def test_ragged_multi_tile(G, orc, geom):
    T = geom["tile"]
    for mix in MIXES:
        for size in (T - 1, T, T + 1, 3 * T + 7, 7 * T - 3):
            b = make_buffer(mix, size, seed=size)
            check_utf8(G, orc, b.data, label=f"{geom['index']} {mix} {size}")
            bi = make_buffer(mix, size, seed=size, error_rate=5e-5, error_seed=size + 1)
            check_utf8(G, orc, bi.data, label=f"{geom['index']} {mix} {size} invalid")
            b16 = make_buffer(mix, size - size % 2, seed=size, encoding="utf-16-le")
            check_utf16(G, orc, b16.data, label=f"{geom['index']} {mix} {size} utf16")
            bi16 = make_buffer(mix, size - size % 2, seed=size, encoding="utf-16-le", error_rate=5e-5,
                               error_seed=size + 2)
            check_utf16(G, orc, bi16.data, label=f"{geom['index']} {mix} {size} utf16 invalid")


@pytest.mark.parametrize("filler", ["ascii", "emoji"])
def test_boundary_straddle(G, orc, geom, filler):
    pats = _utf8_patterns()
    for bnd in (1024, geom["wave"], geom["tile"], 2 * geom["tile"]):
        for delta in range(-4, 5):
            pos = bnd + delta
            for p in pats:
                data = _filler(filler, pos) + p + _filler(filler, 37)
                check_utf8(G, orc, np.frombuffer(data, dtype=np.uint8), label=f"{bnd}{delta:+d} {p.hex()}")
    fill = np.frombuffer({"ascii": "a", "emoji": "\U0001f600"}[filler].encode("utf-16-le"), dtype="<u2")
    pats16 = [np.array(x, dtype=np.uint16) for x in ([0xD800], [0xDC00], [0xDC00, 0xD800], [0xD83D, 0xDE00],
                                                     [0x20AC], [0xD83D, 0xD83D, 0xDE00])]
    for bnd in (512, geom["wave"] // 2, geom["tile"] // 2, geom["tile"]):
        for delta in range(-3, 4):
            pos = bnd + delta
            k = pos // fill.size
            pre = np.concatenate([np.tile(fill, k), np.full(pos - k * fill.size, 0x61, dtype=np.uint16)])
            for p in pats16:
                check_utf16(G, orc, np.concatenate([pre, p, np.tile(fill, 9)]).astype(np.uint16),
                            label=f"{bnd}{delta:+d} {p}")


def test_random_bytes(G, orc, geom):
    rng = np.random.default_rng(100 + geom["index"])
    T = geom["tile"]
    for n in (5000, T, 3 * T + 5):
        check_utf8(G, orc, rng.integers(0, 256, size=n, dtype=np.uint8), label=f"random {n}")
        check_utf8(G, orc, rng.integers(0xF0, 0x100, size=n, dtype=np.uint8), label=f"high {n}")
        check_utf16(G, orc, rng.integers(0xD700, 0xE100, size=n // 2).astype(np.uint16), label=f"sur {n}")


def test_batches(G, orc, geom):
    for mix in ("mix1m", "cjk", "emoji"):
        for median in (3, 40, 700):
            b = make_batch(k=600, seed=SEED_BATCH + 11 + median, median=median, sigma=1.2, lo=0, hi=40_000,
                           error_fraction=0.2, mixes=(mix,))
            check_batch(G, orc, b.data, b.offsets, label=f"{geom['index']} {mix}/{median}")
            b16 = make_batch(k=600, seed=SEED_BATCH + 31 + median, encoding="utf-16-le", median=median, sigma=1.2,
                             lo=0, hi=40_000, error_fraction=0.2, mixes=(mix,))
            check_batch16(G, orc, b16.data, b16.offsets, label=f"{geom['index']} {mix}/{median} utf16")
    b = make_batch(k=3000, seed=SEED_BATCH + 3, median=120, sigma=1.5, lo=0, hi=100_000, error_fraction=0.05)
    total = int(orc.convert_utf8_to_utf16le_batch(b.data, b.offsets)[3][-1])
    for in_off, cap in ((0, None), (7, None), (0, total // 3)):
        check_batch(G, orc, b.data, b.offsets, in_off=in_off, cap=cap, label=f"{geom['index']} off{in_off}")


def test_batch_stage_overflow(G, orc, geom):
    rng = np.random.default_rng(3)
    strings = []
    for _ in range(100):
        strings.append(b"\xf5" * int(rng.integers(200, 3000)))
        strings.append(random_text(rng, "emoji", int(rng.integers(1, 60))).tobytes())
        strings.append(random_text(rng, "mix1m", int(rng.integers(1, 60))).tobytes())
    data, offsets = pack(strings)
    st = check_batch(G, orc, data, offsets, label="overflow")
    assert np.all(st[0::3] == O.TOO_SHORT) and np.all(st[1::3] == O.OK)
    # single buffer: a run of F5 bytes longer than a wave's stage
    check_utf8(G, orc, np.frombuffer(b"ab" + b"\xf5" * (3 * geom["wave"]) + "€".encode() * 50, np.uint8),
               label="f5 run")


def test_tuner_table_and_parity(G, orc, tmp_path):
    from paper_2111_08692_amd import tune as T
    sample = make_buffer("mix1m", 1 << 20, seed=5).data
    sizes = (1 << 15, 1 << 18, 1 << 21)
    T.reset()
    shipped = [[(G.get_geometry(op, c), G.get_schedule(op, c)) for c in range(G.SIZE_CLASSES)]
               for op in range(G.OP_COUNT)]
    try:
        res = T.tune(sample, sizes=sizes, min_ms=0.3, reps=2)
        names = T.geometry_names()
        assert res["geometries"] == names and res["schedules"] == list(G.SCHEDULE_NAMES)
        assert len(res["candidates"]) == 2 * len(names)
        assert set(res["table"]) == set(T.OPS) and set(res["schedule"]) == set(T.OPS)
        for op, rows in res["measured"].items():
            assert len(rows) == len(sizes)
            for r in rows:
                assert len(r["us"]) == len(res["candidates"]) and min(r["us"]) > 0
                assert r["choice"] in res["candidates"]
        # installed: the library reports the tables' choices
        for op, row in res["table"].items():
            assert len(row) == G.SIZE_CLASSES
            for c in (0, 15, 18, 21, 40):
                assert G.get_geometry(T.OPS[op], c) == names.index(row[c])
                assert G.get_schedule(T.OPS[op], c) == G.SCHEDULE_NAMES.index(res["schedule"][op][c])
        # results under the tuned table equal the oracle's
        for n in (30_000, 250_000, 2_000_000):
            b = make_buffer("mix1m", n, seed=n, error_rate=1e-5, error_seed=n + 1)
            check_utf8(G, orc, b.data, label=f"tuned {n}")
            b16 = make_buffer("cjk", n, seed=n, encoding="utf-16-le")
            check_utf16(G, orc, b16.data, label=f"tuned16 {n}")
        bb = make_batch(k=800, seed=SEED_BATCH + 1, median=300, sigma=1.0, lo=0, hi=20_000, error_fraction=0.1)
        check_batch(G, orc, bb.data, bb.offsets, label="tuned batch")
        # JSON round trip
        path = tmp_path / "tune.json"
        T.save(res, str(path))
        T.reset()
        assert [[(G.get_geometry(op, c), G.get_schedule(op, c)) for c in range(G.SIZE_CLASSES)]
                for op in range(G.OP_COUNT)] == shipped
        again = T.apply_file(str(path))
        assert again["table"] == res["table"] and again["schedule"] == res["schedule"]
        for op, row in res["table"].items():
            assert [names[G.get_geometry(T.OPS[op], c)] for c in range(G.SIZE_CLASSES)] == row
            assert [G.SCHEDULE_NAMES[G.get_schedule(T.OPS[op], c)] for c in range(G.SIZE_CLASSES)] \
                == res["schedule"][op]
    finally:
        T.reset()


def test_tuner_command_line(G, tmp_path):
    """``python -m paper_2111_08692_amd.tune`` (its main(), in this process):
    a file of text in, a JSON table out that installs again."""
    from paper_2111_08692_amd import tune as T
    text = tmp_path / "corpus.txt"
    text.write_bytes(make_buffer("cyrillic", 300_000, seed=9).data.tobytes())
    out = tmp_path / "t.json"
    try:
        assert T.main([str(text), "-o", str(out), "--ops", "convert_utf8_to_utf16le,validate_utf16le",
                       "--sizes", "40000,400000"]) == 0
        res = T.apply_file(str(out))
        assert set(res["table"]) == {"convert_utf8_to_utf16le", "validate_utf16le"}
        assert [r["bytes"] <= 400000 for r in res["measured"]["validate_utf16le"]] == [True, True]
    finally:
        T.reset()
