"""The call epoch that tags look-back status words wraps on the device:
the finalize kernel of the call that reaches the epoch period clears every
status word of its workspace.  With UTFGPU_EPOCH_PERIOD=3 (read once per
process, so in a child process) the epoch wraps every second call; large
calls that leave many status words, small calls, validate calls and
replays of a captured graph are interleaved so that a stale word of an
earlier call meets the current epoch at every offset of the cycle.  Every
result must equal the oracle's."""
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


def test_epoch_wrap_matches_oracle():
    env = dict(os.environ, UTFGPU_EPOCH_PERIOD="3")
    r = subprocess.run([sys.executable, "-c", "ROOT_DIR = " + repr(ROOT) + "\n" + CHILD], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "epoch wrap ok" in r.stdout
