"""Host logic of the serving loop: the output-pool ring (no GPU)."""
import pytest

from paper_2111_08692_amd.serve import _Ring


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


def test_ring_rejects_oversize():
    with pytest.raises(ValueError):
        _Ring(10).alloc(11)
