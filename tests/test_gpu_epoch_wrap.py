"""The call epoch that tags look-back status words wraps on the device:
the last kernel of the call that reaches the epoch period (the finalize
kernel, or the post kernel of a batched call) clears every status word of
its workspace.  With UTFGPU_EPOCH_PERIOD=3 (read once per process, so in a
child process) the epoch wraps every second call; large calls that leave
many status words, small calls, validate calls, batched calls in both
directions and replays of a captured graph are interleaved so that a stale
word of an earlier call meets the current epoch at every offset of the
cycle, in block and in ticket tile order.  Every result must equal the
oracle's."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import sys
sys.path.insert(0, ROOT_DIR)
import numpy as np, torch
import oracle as O
import paper_2111_08692_amd as G
from workloads import make_buffer

def check8(d, host, out, label):
    st, cnt, _ = G.convert_utf8_to_utf16le(d, out=out)
    ost, ocnt, oout = O.convert_utf8_to_utf16le(host)
    assert (st, cnt) == (ost, ocnt), label
    assert np.array_equal(out[:cnt].cpu().numpy().view(np.uint16), oout[:ocnt]), label

X = make_buffer("emoji", 3 << 20, seed=11).data
Y = make_buffer("cjk", 3 << 20, seed=12).data
Z = make_buffer("ascii", 4096, seed=13).data
dx, dy, dz = (torch.from_numpy(a).to("cuda") for a in (X, Y, Z))
out = torch.empty(3 << 20, dtype=torch.int16, device="cuda")
small = torch.empty(4096, dtype=torch.int16, device="cuda")
for n_small in range(7):
    check8(dx, X, out, ("x", n_small))
    for i in range(n_small):
        assert G.convert_utf8_to_utf16le(dz, out=small)[:2] == (0, 4096)
        if i % 2:
            assert G.validate_utf8(dy) == (0, Y.size)
    check8(dy, Y, out, ("y", n_small))
    # the reverse direction on the same workspace
    u = torch.from_numpy(O.convert_utf8_to_utf16le(X)[2][:O.utf16_length_from_utf8(X)].view(np.int16)).to("cuda")
    st, cnt, back = G.convert_utf16le_to_utf8(u)
    assert (st, cnt) == (0, X.size) and np.array_equal(back[:cnt].cpu().numpy(), X), ("16to8", n_small)

# batched calls (whose post kernel ends the call) between single-buffer calls
from workloads.mixes import make_batch

def check_batch(bt, enc, label):
    k = bt.offsets.size - 1
    offs = torch.from_numpy(bt.offsets).to("cuda")
    oo = torch.empty(k + 1, dtype=torch.int64, device="cuda")
    rs = G.results_tensor(k)
    if enc == "utf-8":
        d = torch.from_numpy(bt.data).to("cuda")
        o = torch.empty(2 * bt.data.size, dtype=torch.int16, device="cuda")
        assert G.convert_utf8_to_utf16le_batch_async(d, offs, o, oo, rs) == 0
        ost, ocnt, oout, ooff = O.convert_utf8_to_utf16le_batch(bt.data, bt.offsets)
        got = o.cpu().numpy().view(np.uint16)
    else:
        d = torch.from_numpy(bt.data.view(np.int16)).to("cuda")
        o = torch.empty(3 * bt.data.size, dtype=torch.uint8, device="cuda")
        assert G.convert_utf16le_to_utf8_batch_async(d, offs, o, oo, rs) == 0
        ost, ocnt, oout, ooff = O.convert_utf16le_to_utf8_batch(bt.data, bt.offsets)
        got = o.cpu().numpy()
    torch.cuda.synchronize()
    st, cnt = G.decode_results(rs, k)
    assert np.array_equal(oo.cpu().numpy(), ooff), label
    assert np.array_equal(st, ost) and np.array_equal(cnt, ocnt), label
    valid = np.repeat(ost == O.OK, np.diff(ooff))
    assert np.array_equal(got[:ooff[-1]][valid], oout[valid]), label

b8 = make_batch(k=1500, seed=41, median=2000, sigma=1.0, lo=0, hi=50_000, error_fraction=0.05)
b16 = make_batch(k=1500, seed=42, encoding="utf-16-le", median=2000, sigma=1.0, lo=0, hi=50_000, error_fraction=0.05)
for rep in range(6):
    check_batch(b8, "utf-8", ("batch8", rep))
    for i in range(rep % 3):
        assert G.convert_utf8_to_utf16le(dz, out=small)[:2] == (0, 4096)
    check_batch(b16, "utf-16-le", ("batch16", rep))
    check8(dx, X, out, ("x after batches", rep))

# a captured call replayed past many wraps, eager calls on the same stream between replays
s = torch.cuda.Stream()
res = G.result_tensor()
with torch.cuda.stream(s):
    assert G.convert_utf8_to_utf16le_async(dy, out, res, stream=s) == 0   # workspace sized before capture
s.synchronize()
g = torch.cuda.CUDAGraph()
with torch.cuda.graph(g, stream=s):
    assert G.convert_utf8_to_utf16le_async(dy, out, res, stream=s) == 0
ost, ocnt, oout = O.convert_utf8_to_utf16le(Y)
other = torch.empty(3 << 20, dtype=torch.int16, device="cuda")
for rep in range(9):
    with torch.cuda.stream(s):
        for i in range(rep % 3):
            assert G.convert_utf8_to_utf16le(dx, out=other, stream=s)[:2] == (0, O.utf16_length_from_utf8(X))
        out.fill_(0x5A)
    s.synchronize()
    g.replay()
    torch.cuda.synchronize()
    assert G.decode_result(res) == (ost, ocnt), ("replay", rep)
    assert np.array_equal(out[:ocnt].cpu().numpy().view(np.uint16), oout[:ocnt]), ("replay", rep)
print("epoch wrap ok", flush=True)
'''


@pytest.mark.parametrize("schedule", ["0", "1"], ids=["block", "ticket"])
def test_epoch_wrap_matches_oracle(schedule):
    env = dict(os.environ, UTFGPU_EPOCH_PERIOD="3", UTFGPU_SCHEDULE=schedule)
    r = subprocess.run([sys.executable, "-c", "ROOT_DIR = " + repr(ROOT) + "\n" + CHILD], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "epoch wrap ok" in r.stdout
