"""Serving loop: every request's result in the mix equals its result alone
(the single-buffer call on the same payload) and the oracle's, bit-exact,
including the outputs of valid requests; at a reduced shape and at the
serving workload's own shape (10 000 requests up to 16 MiB, four streams,
batches up to 256 MiB), open loop and all at once; admission by arena space
holds requests back under a small HBM budget."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import make_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2111_08692_amd as G
    G.load()
    return G


@pytest.fixture(scope="module")
def served(G):
    from paper_2111_08692_amd.serve import Server
    reqs = make_requests(1500, rate=50_000, median=2048, hi=256 << 10, invalid_fraction=0.05,
                         pool_bytes=4 << 20)
    srv = Server(reqs, nstreams=3, hbm_budget=_everything(reqs), max_batch_bytes=1 << 20)
    srv.prewarm()
    res = srv.run(collect=True)
    return reqs, srv, res


def _everything(reqs):
    """An arena budget that holds every request's reservation at once (the
    outputs are read as each launch completes)."""
    from paper_2111_08692_amd.serve import reservation
    return (sum(reservation(0, int(d)) for d in np.diff(reqs.off8)) +
            sum(reservation(1, int(d)) for d in np.diff(reqs.off16)) + (1 << 20))


def payload(reqs, rid):
    if reqs.kind[rid] == 0:
        j = int(np.searchsorted(reqs.ids8, rid))
        return reqs.data8[reqs.off8[j]:reqs.off8[j + 1]]
    j = int(np.searchsorted(reqs.ids16, rid))
    return reqs.data16[reqs.off16[j]:reqs.off16[j + 1]]


def test_results_equal_alone(G, served):
    reqs, srv, res = served
    assert np.all(res.latency > 0) and np.all(np.isfinite(res.latency))
    assert (res.status != 0).sum() > 20 and (res.status == 0).sum() > 1000
    for rid in range(reqs.arrival.size):
        p = payload(reqs, rid)
        if reqs.kind[rid] == 0:
            d = torch.from_numpy(p).cuda()
            st, cnt, out = G.convert_utf8_to_utf16le(d)
        else:
            d = torch.from_numpy(p.view(np.int16)).cuda()
            st, cnt, out = G.convert_utf16le_to_utf8(d)
        assert (res.status[rid], res.count[rid]) == (st, cnt), rid
        if st == 0:
            alone = out[:cnt].cpu().numpy()
            alone = alone.view(np.uint16) if reqs.kind[rid] == 0 else alone
            assert np.array_equal(srv.output_of(res, rid), alone), rid


def test_sample_against_oracle(served, orc):
    reqs, srv, res = served
    rng = np.random.default_rng(0)
    for rid in rng.choice(reqs.arrival.size, size=200, replace=False):
        p = payload(reqs, int(rid))
        if reqs.kind[rid] == 0:
            st, cnt, out = orc.convert_utf8_to_utf16le(p)
        else:
            st, cnt, out = orc.convert_utf16le_to_utf8(p)
        assert (res.status[rid], res.count[rid]) == (st, cnt), rid
        if st == 0:
            assert np.array_equal(srv.output_of(res, int(rid)), out[:cnt]), rid


def test_burst_held_back_by_hbm_budget(G, orc):
    """Everything arrives at once while an artificial HBM budget gives the
    arena room for a few requests only: requests are held back, admitted as
    completions free space, and every result (outputs read as each launch
    completes, before the ring reuses its space) is the oracle's."""
    from paper_2111_08692_amd.serve import Server
    reqs = make_requests(300, rate=50_000, median=4096, hi=64 << 10, invalid_fraction=0.02,
                         pool_bytes=2 << 20, seed=601)
    srv = Server(reqs, nstreams=2, hbm_budget=1 << 20, max_batch_bytes=128 << 10, max_inflight=4)
    assert srv.arena_bytes == 1 << 20 and srv.free_hbm_at_start > 1 << 30
    res = srv.run(time_scale=0.0)
    assert res.held_back > 0 and res.held_passes > 0
    for rid in range(reqs.arrival.size):
        p = payload(reqs, rid)
        if reqs.kind[rid] == 0:
            st, cnt, _ = G.convert_utf8_to_utf16le(torch.from_numpy(p).cuda())
            ost, ocnt, _ = orc.convert_utf8_to_utf16le(p)
        else:
            st, cnt, _ = G.convert_utf16le_to_utf8(torch.from_numpy(p.view(np.int16)).cuda())
            ost, ocnt, _ = orc.convert_utf16le_to_utf8(p)
        assert (res.status[rid], res.count[rid]) == (st, cnt) == (ost, ocnt), rid


def test_budget_too_small_for_a_request(G):
    from paper_2111_08692_amd.serve import Server
    reqs = make_requests(20, median=4096, hi=64 << 10, pool_bytes=2 << 20, seed=602)
    with pytest.raises(ValueError):
        Server(reqs, nstreams=1, hbm_budget=4096)


def test_invalid_request_widens_the_batch(G):
    """An invalid UTF-8 request of bytes >= F0 counts two words per byte;
    the valid requests batched after it must still get their whole output
    (the pool reserves the worst case of any input)."""
    from paper_2111_08692_amd.serve import Server
    from workloads import RequestSet
    p8 = [np.full(500, 0xF5, np.uint8), np.full(3000, 0x61, np.uint8), np.full(3000, 0x62, np.uint8)]
    p16 = [np.full(10, 0x41, np.uint16)]
    off8 = np.r_[0, np.cumsum([p.size for p in p8])].astype(np.int64)
    off16 = np.r_[0, np.cumsum([p.size for p in p16])].astype(np.int64)
    reqs = RequestSet(arrival=np.zeros(4), kind=np.array([0, 0, 0, 1], np.int8),
                      size=np.array([500, 3000, 3000, 20]), mixes=["ascii"] * 4,
                      invalid=np.array([True, False, False, False]), ids8=np.array([0, 1, 2]), off8=off8,
                      data8=np.concatenate(p8), ids16=np.array([3]), off16=off16, data16=np.concatenate(p16))
    srv = Server(reqs, nstreams=1, hbm_budget=1 << 20)
    res = srv.run(time_scale=0.0, collect=True)
    assert list(res.status) == [1, 0, 0, 0] and list(res.count[1:]) == [3000, 3000, 10]
    assert np.all(srv.output_of(res, 1) == 0x61) and np.all(srv.output_of(res, 2) == 0x62)


# --------------------------------------------------------------------------
# the serving workload at its own shape
# --------------------------------------------------------------------------

def _oracle_all(orc, reqs):
    """Per request (status, count, output) from the oracle's batched calls
    over each direction's payloads (every request converted on its own)."""
    out = {}
    for kind, ids, data, off in ((0, reqs.ids8, reqs.data8, reqs.off8), (1, reqs.ids16, reqs.data16, reqs.off16)):
        if ids.size == 0:
            continue
        conv = orc.convert_utf8_to_utf16le_batch if kind == 0 else orc.convert_utf16le_to_utf8_batch
        st, cnt, o, oo = conv(data, off)
        for j, rid in enumerate(ids):
            a, c = int(oo[j]), int(cnt[j])
            out[int(rid)] = (int(st[j]), c, o[a:a + c] if st[j] == 0 else None)
    return out


@pytest.fixture(scope="module")
def workload_shape(G, orc):
    from paper_2111_08692_amd.serve import Server
    reqs = make_requests(10_000)   # Poisson 50k/s, median 32 KiB, 64 B..16 MiB, 50/50, 0.5% invalid
    assert reqs.size.max() > (4 << 20) and reqs.invalid.sum() > 20
    srv = Server(reqs, nstreams=4, hbm_budget=_everything(reqs), max_batch_bytes=256 << 20)
    srv.prewarm()
    return reqs, srv, _oracle_all(orc, reqs)


@pytest.mark.parametrize("time_scale", [1.0, 0.0], ids=["open_loop_50k", "burst"])
def test_workload_shape_every_request_vs_oracle(workload_shape, time_scale):
    reqs, srv, ref = workload_shape
    res = srv.run(time_scale=time_scale, collect=True)
    assert res.launches >= 2 and np.all(np.isfinite(res.latency))
    for rid in range(reqs.arrival.size):
        st, cnt, o = ref[rid]
        assert (int(res.status[rid]), int(res.count[rid])) == (st, cnt), rid
        if st == 0:
            assert np.array_equal(srv.output_of(res, rid), o), rid
