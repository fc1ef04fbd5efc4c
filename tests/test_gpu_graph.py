"""The batched calls captured once in a HIP graph (torch.cuda.CUDAGraph)
and replayed with new input contents and new string boundaries (same sizes)
written between replays; every replay is checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import random_text

pytestmark = pytest.mark.gpu

N8, K = 200_000, 3000


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2111_08692_amd as G
    G.load()
    return G


def replay_input(seed, n, k, encoding):
    rng = np.random.default_rng(seed)
    t = random_text(rng, "mix1m" if seed % 2 else "emoji", n, encoding=encoding)[:n]
    if t.size < n:
        t = np.concatenate([t, np.full(n - t.size, 0x20, dtype=t.dtype)])
    cuts = np.sort(rng.choice(np.arange(1, n), size=k - 1, replace=False))
    offsets = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    if seed % 3 == 0:   # some empty strings
        offsets[5:9] = offsets[5]
    return t, offsets


@pytest.mark.parametrize("direction", ["8to16", "16to8"])
def test_graph_replays(G, orc, direction):
    to16 = direction == "8to16"
    n = N8 if to16 else N8 // 2
    s = torch.cuda.Stream()
    if to16:
        d = torch.zeros(n, dtype=torch.uint8, device="cuda")
        out = torch.zeros(2 * n, dtype=torch.int16, device="cuda")
        call = G.convert_utf8_to_utf16le_batch_async
        enc, oracle_call = "utf-8", orc.convert_utf8_to_utf16le_batch
    else:
        d = torch.zeros(n, dtype=torch.int16, device="cuda")
        out = torch.zeros(3 * n, dtype=torch.uint8, device="cuda")
        call = G.convert_utf16le_to_utf8_batch_async
        enc, oracle_call = "utf-16-le", orc.convert_utf16le_to_utf8_batch
    offs = torch.zeros(K + 1, dtype=torch.int64, device="cuda")
    oo = torch.zeros(K + 1, dtype=torch.int64, device="cuda")
    res = G.results_tensor(K)

    def load(seed):
        t, o = replay_input(seed, n, K, enc)
        d.copy_(torch.from_numpy(t if to16 else t.view(np.int16)))
        offs.copy_(torch.from_numpy(o))
        torch.cuda.synchronize()
        return t, o

    def check(t, o, label):
        ost, ocnt, oout, ooff = oracle_call(t, o)
        st, cnt = G.decode_results(res, K)
        assert np.array_equal(oo.cpu().numpy(), ooff), label
        assert np.array_equal(st, ost) and np.array_equal(cnt, ocnt), label
        got = out.cpu().numpy()
        got = got.view(np.uint16) if to16 else got
        valid = np.repeat(ost == O.OK, np.diff(ooff))
        total = int(ooff[-1])
        assert np.array_equal(got[:total][valid], oout[valid]), label

    t, o = load(1)
    with torch.cuda.stream(s):   # the capture stream's workspace exists and is large enough
        assert call(d, offs, out, oo, res, stream=s) == 0
    s.synchronize()
    check(t, o, "eager")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        assert call(d, offs, out, oo, res, stream=s) == 0
    for rep in range(2, 7):
        t, o = load(rep)
        out.fill_(0x5A)   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(t, o, f"replay {rep}")
