"""GPU parity at the benchmark's full size (1 GiB per buffer), in the same
launch configuration the benchmark times.

Each buffer is checked element by element:
* a valid buffer: status, count and every output unit against the oracle's
  conversion of the whole buffer;
* an invalid buffer: the first error (position and kind) against what the
  generator injected and against the oracle, and every output unit of the
  valid prefix against the oracle's conversion of that prefix;
* the output length against the oracle's length query over the whole
  buffer, validate-only against the oracle, and the round trip
  UTF-8 -> UTF-16LE -> UTF-8 (and back) on the device.
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


def _check_all_utf8(orc, data, gpu_out, limit):
    """Every output word of the valid prefix data[:limit] (the whole buffer
    when it is valid)."""
    st, cnt, ref = orc.convert_utf8_to_utf16le(data[:limit])
    assert st == 0
    got = to_host(gpu_out, cnt)
    assert got.size == cnt
    if not np.array_equal(got, ref[:cnt]):
        bad = int(np.nonzero(got != ref[:cnt])[0][0])
        raise AssertionError(f"output word {bad}: device {got[bad]:#x}, oracle {ref[bad]:#x}")


def _check_all_utf16(orc, data, gpu_out, limit):
    st, cnt, ref = orc.convert_utf16le_to_utf8(data[:limit])
    assert st == 0
    got = to_host(gpu_out, cnt)
    assert got.size == cnt
    if not np.array_equal(got, ref[:cnt]):
        bad = int(np.nonzero(got != ref[:cnt])[0][0])
        raise AssertionError(f"output byte {bad}: device {got[bad]:#x}, oracle {ref[bad]:#x}")


@pytest.mark.parametrize("mix", SCRIPT_MIXES)
def test_fullsize_utf8(G, orc, pool, mix):
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
            _check_all_utf8(orc, data, out, SIZE)
            back = torch.empty(SIZE, dtype=torch.uint8, device="cuda")
            st2, cnt2, _ = G.convert_utf16le_to_utf8(out[:cnt], out=back)
            assert (st2, cnt2) == (0, SIZE) and torch.equal(back, d)
        else:
            e = b.first_error
            assert len(b.errors) > 500
            ost, oe = orc.validate_utf8(data[:e + 8])
            assert (st, cnt) == (vst, vcnt) == (ost, oe) and oe == e
            assert orc.validate_utf8(data) == (ost, oe)
            _check_all_utf8(orc, data, out, e)
        del d, out


@pytest.mark.parametrize("mix", SCRIPT_MIXES)
def test_fullsize_utf16(G, orc, pool, mix):
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
            _check_all_utf16(orc, data, out, m)
            back = torch.empty(m, dtype=torch.int16, device="cuda")
            st2, cnt2, _ = G.convert_utf8_to_utf16le(out[:cnt], out=back)
            assert (st2, cnt2) == (0, m) and torch.equal(back, d)
        else:
            e = b.first_error
            assert len(b.errors) > 250
            ost, oe = orc.validate_utf16le(data[:e + 4])
            assert (st, cnt) == (vst, vcnt) == (ost, oe) and oe == e
            assert orc.validate_utf16le(data) == (ost, oe)
            _check_all_utf16(orc, data, out, e)
        del d, out
