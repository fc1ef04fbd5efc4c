"""Host logic of the serving loop: the output-pool ring and the windows
that pre-size the library's workspaces (no GPU)."""
import numpy as np
import pytest

from paper_2111_08692_amd.serve import ALIGN, _Ring, prewarm_windows, reservation


def test_ring_alloc_free_wrap():
    r = _Ring(100)
    a = r.alloc(40)
    b = r.alloc(40)
    assert a == (0, 40) and b == (40, 40)
    assert r.alloc(30) is None            # 20 left at the end, 0 at the start
    r.free(40)                            # first one done
    c = r.alloc(30)                       # does not fit before the end: starts over, charged the 20 skipped
    assert c == (0, 50)
    r.free(40)
    r.free(50)
    assert r.used == 0


def test_ring_empty_starts_over():
    """Once everything is freed the next reservation may take the whole
    ring, wherever the last one ended."""
    r = _Ring(100)
    assert r.alloc(50) == (0, 50)
    r.free(50)
    assert r.head == 0 and r.used == 0
    assert r.alloc(60) == (0, 60)
    r.free(60)
    assert r.alloc(100) == (0, 100)


def test_reservation_is_aligned_worst_case():
    assert reservation(0, 1) == ALIGN and reservation(0, 64) == 256 and reservation(0, 65) == 512
    assert reservation(1, 100) == 512 and reservation(1, 85) == 256 and reservation(1, 0) == 0


def test_ring_rejects_oversize():
    with pytest.raises(ValueError):
        _Ring(10).alloc(11)


def _formable(off, kind, max_batch, pool):
    """Every batch the scheduler can form with all requests arrived: from
    each i, the window up to the batch limit, halved while its output
    reservation exceeds the pool (as the scheduler does for a full ring)."""
    per_unit = 4 if kind == 0 else 3
    nq = off.size - 1
    for i in range(nq):
        j = max(int(np.searchsorted(off, off[i] + max_batch // (1 + kind), side="right")) - 1, i + 1)
        while True:
            if per_unit * int(off[j] - off[i]) <= pool:
                yield i, j
            if j == i + 1:
                break
            j = i + (j - i) // 2


@pytest.mark.parametrize("seed", range(6))
def test_prewarm_windows_bound_every_batch(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    sizes = np.exp(rng.normal(np.log(200), 1.5, size=n)).astype(np.int64) + 1
    off = np.concatenate([[0], np.cumsum(sizes)])
    for kind in (0, 1):
        max_batch = int(rng.integers(50, 20_000))
        pool = int(rng.integers(100, 40_000))
        wins = prewarm_windows(off, kind, max_batch, pool)
        per_unit = 4 if kind == 0 else 3
        formable = list(_formable(off, kind, max_batch, pool))
        if not formable:
            assert wins == []
            continue
        assert 1 <= len(wins) <= 2
        for i, j in wins:   # each is a call the pool can hold
            assert 0 <= i < j <= n and per_unit * int(off[j] - off[i]) <= pool
        assert max(int(off[j] - off[i]) for i, j in wins) >= max(int(off[j] - off[i]) for i, j in formable)
        assert max(j - i for i, j in wins) >= max(j - i for i, j in formable)
