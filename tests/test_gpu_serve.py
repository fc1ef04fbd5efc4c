"""Serving loop: every request's result in the mix equals its result alone
(the single-buffer call on the same payload) and, on a sample, the oracle's;
bit-exact, including the outputs of valid requests."""
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
    bound = max(4 * reqs.data8.size, 3 * reqs.data16.size) + (1 << 20)
    srv = Server(reqs, nstreams=3, pool_bytes=bound, max_batch_bytes=1 << 20)
    srv.prewarm()
    res = srv.run()
    return reqs, srv, res


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


def test_burst_and_tight_pool(G):
    """Everything arrives at once into a pool that holds a few requests:
    admission has to wait for completions, results stay exact."""
    from paper_2111_08692_amd.serve import Server
    reqs = make_requests(300, rate=50_000, median=4096, hi=64 << 10, invalid_fraction=0.02,
                         pool_bytes=2 << 20, seed=601)
    srv = Server(reqs, nstreams=2, pool_bytes=1 << 20, max_batch_bytes=128 << 10, max_inflight=4)
    res = srv.run(time_scale=0.0)
    for rid in range(reqs.arrival.size):
        p = payload(reqs, rid)
        if reqs.kind[rid] == 0:
            st, cnt, _ = G.convert_utf8_to_utf16le(torch.from_numpy(p).cuda())
        else:
            st, cnt, _ = G.convert_utf16le_to_utf8(torch.from_numpy(p.view(np.int16)).cuda())
        assert (res.status[rid], res.count[rid]) == (st, cnt), rid


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
    srv = Server(reqs, nstreams=1, pool_bytes=1 << 20)
    res = srv.run(time_scale=0.0)
    assert list(res.status) == [1, 0, 0, 0] and list(res.count[1:]) == [3000, 3000, 10]
    assert np.all(srv.output_of(res, 1) == 0x61) and np.all(srv.output_of(res, 2) == 0x62)
