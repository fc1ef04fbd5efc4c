"""CPU checks of the geometry and scan-schedule tuning tables and the
tuner's host logic: the table calls of the C ABI (host state, no GPU), size
classes, argument checks, the table fill and choice rules, the candidate
list, the character-boundary cuts of the tuner's inputs, and installing /
refusing a saved table."""
import json
import os

import numpy as np
import pytest


@pytest.fixture(scope="module")
def G():
    import paper_2111_08692_amd as G
    if not os.path.exists(G.LIB_PATH):
        from paper_2111_08692_amd.build import build
        build()
    G.load()
    yield G
    for op in range(G.OP_COUNT):
        for c in range(G.SIZE_CLASSES):
            G.set_geometry(op, c, -1)
            G.set_schedule(op, c, -1)


@pytest.fixture(scope="module")
def T(G):
    from paper_2111_08692_amd import tune
    return tune


def test_geometries(G):
    geo = G.geometries()
    assert len(geo) >= 2
    assert geo[0] == (8, 4, 32768) and G.tile_bytes() == 32768
    for w, r, tb in geo:
        assert tb == w * r * 1024 and r % 2 == 0 and w * 64 <= 1024
        assert 3 * tb // 2 <= 65536   # 16-bit block offsets of batched UTF-16 calls
    assert len(set(geo)) == len(geo)


def test_size_class_is_ceil_log2(G):
    assert G.size_class(0) == 0 and G.size_class(1) == 0
    for b in (2, 3, 4, 5, 1000, 1 << 20, (1 << 20) + 1, (1 << 40) - 1, 1 << 40):
        assert G.size_class(b) == (b - 1).bit_length(), b
    assert G.size_class((1 << 64) - 1) == G.SIZE_CLASSES - 1


def test_shipped_defaults(G):
    names = [f"{w}x{r}" for w, r, _ in G.geometries()]
    g0, g4x2, g4x4 = 0, names.index("4x2"), names.index("4x4")
    for op in range(G.OP_COUNT):
        for c in range(G.SIZE_CLASSES):
            G.set_geometry(op, c, -1)
    want = {
        G.OP_VALIDATE_UTF8: lambda c: g0,
        G.OP_VALIDATE_UTF16LE: lambda c: g0,
        G.OP_CONVERT_UTF8: lambda c: g4x2 if c <= 22 else g0,
        G.OP_CONVERT_UTF16LE: lambda c: g4x2 if c <= 22 else g0,
        G.OP_BATCH_UTF16LE: lambda c: g4x2 if c <= 22 else g4x4,
        G.OP_BATCH_UTF8: lambda c: g4x2 if c <= 24 else g0,
    }
    for op, f in want.items():
        assert [G.get_geometry(op, c) for c in range(G.SIZE_CLASSES)] == [f(c) for c in range(G.SIZE_CLASSES)], op


def test_set_get_and_argument_checks(G):
    ng = len(G.geometries())
    shipped20 = G.get_geometry(G.OP_CONVERT_UTF8, 20)
    shipped21 = G.get_geometry(G.OP_CONVERT_UTF8, 21)
    other = (shipped20 + 1) % ng
    assert G.set_geometry(G.OP_CONVERT_UTF8, 20, other) == G.OK
    assert G.get_geometry(G.OP_CONVERT_UTF8, 20) == other
    # other operations and classes are untouched
    assert G.get_geometry(G.OP_CONVERT_UTF8, 21) == shipped21 and G.get_geometry(G.OP_VALIDATE_UTF8, 20) == 0
    assert G.set_geometry(G.OP_CONVERT_UTF8, 20, -1) == G.OK
    assert G.get_geometry(G.OP_CONVERT_UTF8, 20) == shipped20
    for op, c, g in ((-1, 0, 0), (G.OP_COUNT, 0, 0), (0, -1, 0), (0, G.SIZE_CLASSES, 0), (0, 0, ng), (0, 0, -2)):
        assert G.set_geometry(op, c, g) == G.ERR_ARG, (op, c, g)
    assert G.get_geometry(G.OP_COUNT, 0) == G.ERR_ARG and G.get_geometry(0, G.SIZE_CLASSES) == G.ERR_ARG
    assert G.load().utfgpu_geometry(ng, None, None, None) == G.ERR_ARG


def test_schedules_shipped_set_get_and_argument_checks(G):
    assert (G.SCHEDULE_BLOCK, G.SCHEDULE_TICKET) == (0, 1) and G.SCHEDULE_NAMES == ("block", "ticket")
    for op in range(G.OP_COUNT):
        for c in range(G.SIZE_CLASSES):
            assert G.set_schedule(op, c, -1) == G.OK
    # shipped: block order for every operation and class
    assert all(G.get_schedule(op, c) == G.SCHEDULE_BLOCK for op in range(G.OP_COUNT) for c in range(G.SIZE_CLASSES))
    g = G.get_geometry(G.OP_BATCH_UTF16LE, 27)
    assert G.set_schedule(G.OP_BATCH_UTF16LE, 27, G.SCHEDULE_TICKET) == G.OK
    assert G.get_schedule(G.OP_BATCH_UTF16LE, 27) == G.SCHEDULE_TICKET
    # the geometry and the other entries are untouched
    assert G.get_geometry(G.OP_BATCH_UTF16LE, 27) == g
    assert G.get_schedule(G.OP_BATCH_UTF16LE, 26) == 0 and G.get_schedule(G.OP_BATCH_UTF8, 27) == 0
    assert G.set_schedule(G.OP_BATCH_UTF16LE, 27, -1) == G.OK and G.get_schedule(G.OP_BATCH_UTF16LE, 27) == 0
    for op, c, v in ((-1, 0, 0), (G.OP_COUNT, 0, 0), (0, -1, 0), (0, G.SIZE_CLASSES, 0), (0, 0, 2), (0, 0, -2)):
        assert G.set_schedule(op, c, v) == G.ERR_ARG, (op, c, v)
    assert G.get_schedule(G.OP_COUNT, 0) == G.ERR_ARG and G.get_schedule(0, G.SIZE_CLASSES) == G.ERR_ARG


def test_candidates(T, G):
    ng = len(G.geometries())
    c = T.candidates()
    assert c[0] == (0, 0) and len(c) == 2 * ng and len(set(c)) == len(c)
    assert set(c) == {(g, s) for g in range(ng) for s in (0, 1)}
    assert T.candidates(False) == [(g, 0) for g in range(ng)]
    names = T.geometry_names()
    assert T.candidate_name(0, 1, names) == names[0] + "/ticket"


def test_choose_and_fill(T):
    assert T.choose([10.0, 9.0, 11.0], 0.03) == 1
    assert T.choose([10.0, 9.8, 11.0], 0.03) == 0   # within the margin: the current geometry stays
    assert T.choose([10.0, 10.5, 11.0], 0.0) == 0
    assert T.choose([10.0, 9.0, 8.9], 0.03, current=2) == 2
    assert T.choose([8.0, 9.0, 8.9], 0.03, current=2) == 0
    row = T.nearest_fill({16: 2, 20: -1, 24: 1}, 30)
    assert row[:19] == [2] * 19 and row[19:23] == [-1] * 4 and row[23:] == [1] * 7
    assert row[18] == 2 and row[22] == -1   # ties go to the smaller class
    assert T.nearest_fill({}, 5) == [-1] * 5


def test_input_cuts_keep_characters_whole(T):
    rng = np.random.default_rng(1)
    text = "".join(rng.choice(list("aé€中😀")) for _ in range(3000))
    u8 = np.frombuffer(text.encode(), dtype=np.uint8)
    u16 = np.frombuffer(text.encode("utf-16-le"), dtype=np.uint16)
    for n in range(0, 200):
        bytes(T._cut_utf8(u8, n)).decode("utf-8")
        assert T._cut_utf8(u8, n).size >= n - 3
        bytes(T._cut_utf16(u16, n).astype("<u2")).decode("utf-16-le")
    for per in (1, 5, 64, 1000):
        offs = T._string_offsets(u8, per, True)
        assert offs[0] == 0 and offs[-1] == u8.size and np.all(np.diff(offs) > 0)
        for a, b in zip(offs[:-1], offs[1:]):
            bytes(u8[a:b]).decode("utf-8")
        offs = T._string_offsets(u16, per, False)
        assert offs[0] == 0 and offs[-1] == u16.size and np.all(np.diff(offs) > 0)
        for a, b in zip(offs[:-1], offs[1:]):
            bytes(u16[a:b].astype("<u2")).decode("utf-16-le")


def _table(T, G, pick):
    names = T.geometry_names()
    return {"library": G.version(), "geometries": names, "schedules": list(G.SCHEDULE_NAMES), "min_gain": 0.03,
            "string_bytes": 4096, "measured": {},
            "table": {op: [names[pick(i, c) % len(names)] for c in range(G.SIZE_CLASSES)]
                      for i, op in enumerate(T.OPS)},
            "schedule": {op: [G.SCHEDULE_NAMES[(i * c) % 2] for c in range(G.SIZE_CLASSES)]
                         for i, op in enumerate(T.OPS)}}


def _state(G):
    return [[(G.get_geometry(op, c), G.get_schedule(op, c)) for c in range(G.SIZE_CLASSES)]
            for op in range(G.OP_COUNT)]


def test_apply_save_load_reset(T, G, tmp_path):
    T.reset()
    shipped = _state(G)
    res = _table(T, G, lambda i, c: i + c)
    path = tmp_path / "t.json"
    T.save(res, str(path))
    T.apply_file(str(path))
    n = len(T.geometry_names())
    for i, op in enumerate(T.OPS):
        for c in range(G.SIZE_CLASSES):
            assert G.get_geometry(T.OPS[op], c) == (i + c) % n
            assert G.get_schedule(T.OPS[op], c) == (i * c) % 2
    T.reset()
    assert _state(G) == shipped


def test_apply_refuses_a_foreign_table(T, G, tmp_path):
    good = _table(T, G, lambda i, c: 1)
    T.reset()
    shipped = _state(G)
    sched_bad = dict(good["schedule"], validate_utf8=["fifo"] * G.SIZE_CLASSES)
    for bad in (dict(good, geometries=good["geometries"][:-1]), dict(good, library="other 9.9"),
                dict(good, schedules=["block"]), dict(good, schedule=sched_bad),
                dict(good, schedule={op: v for op, v in good["schedule"].items() if op != "validate_utf8"}),
                dict(good, table={"no_such_op": good["table"]["validate_utf8"]}),
                dict(good, table={"validate_utf8": good["table"]["validate_utf8"][:10]})):
        path = tmp_path / "bad.json"
        path.write_text(json.dumps(bad))
        with pytest.raises(ValueError):
            T.apply_file(str(path))
        assert _state(G) == shipped   # nothing installed from a refused table
    T.reset()
