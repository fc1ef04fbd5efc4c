"""Host logic of the pipelined host-memory path: chunk cuts (no GPU)."""
import numpy as np

from paper_2111_08692_amd.host_pipeline import cuts_utf8, cuts_utf16
from workloads import random_text


def test_utf8_cuts_at_character_starts():
    rng = np.random.default_rng(1)
    t = random_text(rng, "mix1m", 5000)
    for chunk in (1, 2, 3, 7, 64, 1000):
        c = cuts_utf8(t, chunk)
        assert c[0] == 0 and c[-1] == t.size and all(a < b for a, b in zip(c, c[1:]))
        assert all((t[k] & 0xC0) != 0x80 for k in c[1:-1])
        assert all(b - a <= chunk + 3 for a, b in zip(c, c[1:]))


def test_utf8_cuts_in_long_continuation_runs():
    t = np.array([0x41] + [0x80] * 20 + [0x42], dtype=np.uint8)
    c = cuts_utf8(t, 4)
    assert c[0] == 0 and c[-1] == t.size and all(b - a <= 7 for a, b in zip(c, c[1:]))


def test_utf16_cuts_keep_pairs():
    rng = np.random.default_rng(2)
    t = random_text(rng, "emoji", 4000, encoding="utf-16-le")
    for chunk in (1, 2, 5, 333):
        c = cuts_utf16(t, chunk)
        assert c[0] == 0 and c[-1] == t.size
        assert all(not (0xDC00 <= t[k] <= 0xDFFF) for k in c[1:-1])
