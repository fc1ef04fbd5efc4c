"""GPU parity at the benchmark's full size (1 GiB per buffer), in the same
launch configuration the benchmark times.

The oracle cannot compare 20 GiB quickly, so each buffer is checked by:
* the first error (position and kind) against what the generator injected
  and against the oracle run on the bytes around it;
* output length against the oracle's length query over the whole buffer;
* 24 sampled windows of 64 KiB, each converted by the oracle and compared
  with the GPU output at the offset the oracle's lengths give;
* the round trip UTF-8 -> UTF-16LE -> UTF-8 (and back) on the device.
"""
import multiprocessing as mp
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import torch

import oracle as O
from tests.gpu_util import to_host
from workloads import SCRIPT_MIXES, SEED_UTF8, SEED_UTF8_INVALID, SEED_UTF16, SEED_UTF16_INVALID, make_buffer

pytestmark = pytest.mark.gpu

SIZE = 1 << 30
WIN = 64 << 10
NWIN = 24


@pytest.fixture(scope="module")
def G():
    assert torch.cuda.is_available()
    import paper_2111_08692_amd as G
    G.load()
    return G


@pytest.fixture(scope="module")
def pool():
    ex = ProcessPoolExecutor(max_workers=16, mp_context=mp.get_context("spawn"))
    yield ex
    ex.shutdown()


def _windows(rng, n, char_start):
    """Sorted window starts moved back to a character start."""
    starts = np.sort(rng.integers(0, n - WIN, size=NWIN))
    out = []
    for s in starts:
        s = int(s)
        while s > 0 and not char_start(s):
            s -= 1
        out.append(s)
    return sorted(set(out))


def _check_utf8_windows(G, orc, data, gpu_out, limit, rng):
    """Compare GPU words of sampled windows inside [0, limit)."""
    starts = _windows(rng, limit, lambda s: (data[s] & 0xC0) != 0x80)
    pos, words = 0, 0
    for s in starts:
        words += orc.utf16_length_from_utf8(data[pos:s])
        pos = s
        e = min(s + WIN, limit)
        while e < limit and (data[e] & 0xC0) == 0x80:
            e -= 1
        st, cnt, ref = orc.convert_utf8_to_utf16le(data[s:e])
        assert st == 0
        got = to_host(gpu_out[words:words + cnt], cnt)
        assert np.array_equal(got, ref[:cnt]), ("window", s)


def _check_utf16_windows(G, orc, data, gpu_out, limit, rng):
    starts = _windows(rng, limit, lambda s: not (0xDC00 <= data[s] <= 0xDFFF))
    pos, nbytes = 0, 0
    for s in starts:
        nbytes += orc.utf8_length_from_utf16le(data[pos:s])
        pos = s
        e = min(s + WIN // 2, limit)
        if e < limit and 0xDC00 <= data[e] <= 0xDFFF:
            e -= 1
        st, cnt, ref = orc.convert_utf16le_to_utf8(data[s:e])
        assert st == 0
        got = to_host(gpu_out[nbytes:nbytes + cnt], cnt)
        assert np.array_equal(got, ref[:cnt]), ("window", s)


@pytest.mark.parametrize("mix", SCRIPT_MIXES)
def test_fullsize_utf8(G, orc, pool, mix):
    rng = np.random.default_rng(SEED_UTF8[mix])
    for kind in ("valid", "invalid"):
        rate = 0.0 if kind == "valid" else 1e-6
        b = make_buffer(mix, SIZE, SEED_UTF8[mix], error_rate=rate, error_seed=SEED_UTF8_INVALID[mix],
                        executor=pool)
        data = b.data
        d = torch.from_numpy(data).to("cuda")
        need = orc.utf16_length_from_utf8(data)
        assert G.utf16_length_from_utf8(d) == need
        out = torch.empty(SIZE, dtype=torch.int16, device="cuda")
        res = G.result_tensor()
        assert G.convert_utf8_to_utf16le_async(d, out, res) == 0     # the benchmark's call
        st, cnt = G.decode_result(res)
        vst, vcnt = G.validate_utf8(d)
        if kind == "valid":
            assert (st, cnt) == (0, need) and (vst, vcnt) == (0, SIZE)
            _check_utf8_windows(G, orc, data, out, SIZE, rng)
            back = torch.empty(SIZE, dtype=torch.uint8, device="cuda")
            st2, cnt2, _ = G.convert_utf16le_to_utf8(out[:cnt], out=back)
            assert (st2, cnt2) == (0, SIZE) and torch.equal(back, d)
        else:
            e = b.first_error
            assert len(b.errors) > 500
            ost, oe = orc.validate_utf8(data[:e + 8])
            assert (st, cnt) == (vst, vcnt) == (ost, oe) and oe == e
            _check_utf8_windows(G, orc, data, out, e, rng)
        del d, out


@pytest.mark.parametrize("mix", SCRIPT_MIXES)
def test_fullsize_utf16(G, orc, pool, mix):
    rng = np.random.default_rng(SEED_UTF16[mix])
    m = SIZE // 2
    for kind in ("valid", "invalid"):
        rate = 0.0 if kind == "valid" else 1e-6
        b = make_buffer(mix, SIZE, SEED_UTF16[mix], encoding="utf-16-le", error_rate=rate,
                        error_seed=SEED_UTF16_INVALID[mix], executor=pool)
        data = b.data
        d = torch.from_numpy(data.view(np.int16)).to("cuda")
        need = orc.utf8_length_from_utf16le(data)
        assert G.utf8_length_from_utf16le(d) == need
        out = torch.empty(3 * m, dtype=torch.uint8, device="cuda")
        res = G.result_tensor()
        assert G.convert_utf16le_to_utf8_async(d, out, res) == 0
        st, cnt = G.decode_result(res)
        vst, vcnt = G.validate_utf16le(d)
        if kind == "valid":
            assert (st, cnt) == (0, need) and (vst, vcnt) == (0, m)
            _check_utf16_windows(G, orc, data, out, m, rng)
            back = torch.empty(m, dtype=torch.int16, device="cuda")
            st2, cnt2, _ = G.convert_utf8_to_utf16le(out[:cnt], out=back)
            assert (st2, cnt2) == (0, m) and torch.equal(back, d)
        else:
            e = b.first_error
            assert len(b.errors) > 250
            ost, oe = orc.validate_utf16le(data[:e + 4])
            assert (st, cnt) == (vst, vcnt) == (ost, oe) and oe == e
            _check_utf16_windows(G, orc, data, out, e, rng)
        del d, out
