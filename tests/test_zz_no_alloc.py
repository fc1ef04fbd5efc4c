"""The allocation-free entry point convert_utf8_to_utf16le_noalloc_async,
called through the C ABI, against convert_utf8_to_utf16le_async (the
workspace entry point) and the oracle: bit-exact results and outputs on
consecutive calls, the second with a smaller input, valid and invalid,
at several tile geometries' sizes; and its size limit, checked on the host."""
import ctypes

import numpy as np
import pytest
import torch

from workloads import make_buffer


@pytest.fixture(scope="module")
def G():
    import paper_2111_08692_amd as G
    G.load()
    return G


def test_noalloc_rejects_too_many_tiles(G):
    """2 GiB of input needs 65 537 tiles of 32 KiB: refused before any device
    work (the pointers are never touched)."""
    L = G.load()
    res = ctypes.c_void_p(64)
    assert L.convert_utf8_to_utf16le_noalloc_async(16, 1 << 31, 64, 1 << 31, res, None) == G.ERR_TOO_BIG
    assert L.convert_utf8_to_utf16le_noalloc_async(16, 3, 17, 3, res, None) == G.ERR_ALIGN
    assert L.convert_utf8_to_utf16le_noalloc_async(None, 3, 64, 3, res, None) == G.ERR_NULL
    assert L.convert_utf8_to_utf16le_noalloc_async(16, 3, 64, 3, None, None) == G.ERR_NULL


def _inputs():
    big = make_buffer("emoji", (40 << 20) + 5, seed=71).data          # 32 KiB tiles
    small = make_buffer("cjk", (3 << 20) + 1, seed=72).data           # 8 KiB tiles
    bad = make_buffer("latin", 5 << 20, seed=73, error_rate=2e-6, error_seed=74)
    tiny = make_buffer("mix1m", 777, seed=75).data
    return [("big", big), ("small", small), ("invalid", bad.data), ("tiny", tiny), ("empty", big[:0])]


@pytest.mark.gpu
def test_noalloc_matches_workspace_entry(G, orc):
    cases = _inputs()
    devs = [(name, torch.from_numpy(a).to("cuda"), a) for name, a in cases]
    outs = []
    # consecutive calls on one stream, each smaller than the one before
    for name, d, _ in devs:
        o = torch.full((max(d.numel(), 1),), 0x1234, dtype=torch.int16, device="cuda")
        r = G.result_tensor()
        assert G.convert_utf8_to_utf16le_noalloc_async(d, o, r) == G.OK, name
        outs.append((o, r))
    torch.cuda.synchronize()
    for (name, d, host), (o, r) in zip(devs, outs):
        ref_o = torch.full_like(o, 0x1234)
        ref_r = G.result_tensor()
        assert G.convert_utf8_to_utf16le_async(d, ref_o, ref_r) == G.OK, name
        torch.cuda.synchronize()
        st, cnt = G.decode_result(r)
        assert (st, cnt) == G.decode_result(ref_r), name
        ost, ocnt, oout = orc.convert_utf8_to_utf16le(host)
        assert (st, cnt) == (ost, ocnt), name
        valid = ocnt if ost == 0 else orc.convert_utf8_to_utf16le(host[:ocnt])[1]
        got = o[:valid].cpu().numpy().view(np.uint16)
        assert np.array_equal(got, ref_o[:valid].cpu().numpy().view(np.uint16)), name
        ref = oout[:valid] if ost == 0 else orc.convert_utf8_to_utf16le(host[:ocnt])[2][:valid]
        assert np.array_equal(got, ref), name


@pytest.mark.gpu
def test_noalloc_repeated_small_after_large(G, orc):
    """Many calls in a row reuse the one array; a small call after a large
    one must not see the large one's status words."""
    a = make_buffer("cyrillic", 9 << 20, seed=81).data
    b = make_buffer("emoji", (1 << 20) + 77, seed=82).data
    da, db = torch.from_numpy(a).to("cuda"), torch.from_numpy(b).to("cuda")
    oa = torch.empty(a.size, dtype=torch.int16, device="cuda")
    ob = torch.empty(b.size, dtype=torch.int16, device="cuda")
    ra, rb = G.result_tensor(), G.result_tensor()
    _, na, refa = orc.convert_utf8_to_utf16le(a)
    _, nb, refb = orc.convert_utf8_to_utf16le(b)
    for rep in range(5):
        assert G.convert_utf8_to_utf16le_noalloc_async(da, oa, ra) == G.OK
        assert G.convert_utf8_to_utf16le_noalloc_async(db, ob, rb) == G.OK
        torch.cuda.synchronize()
        assert G.decode_result(ra) == (0, na) and G.decode_result(rb) == (0, nb), rep
        assert np.array_equal(oa[:na].cpu().numpy().view(np.uint16), refa[:na]), rep
        assert np.array_equal(ob[:nb].cpu().numpy().view(np.uint16), refb[:nb]), rep
