"""CPU checks of the C-ABI library: it loads, exports every function that
``include/utfgpu.h`` declares, and its host-only paths (empty input,
argument checks) answer without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "utfgpu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def G():
    import paper_2111_08692_amd as G
    if not os.path.exists(G.LIB_PATH):
        from paper_2111_08692_amd.build import build
        build()
    G.load()
    return G


def test_header_lists_the_api():
    names = declared_functions()
    for n in ("validate_utf8", "validate_utf16le", "utf16_length_from_utf8", "utf8_length_from_utf16le",
              "convert_utf8_to_utf16le", "convert_utf16le_to_utf8"):
        assert n in names


def test_library_exports_every_declared_symbol(G):
    lib = ctypes.CDLL(G.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(G.EXPORTS)


def test_host_only_paths(G):
    L = G.load()
    assert G.version().startswith("utfgpu")
    # empty inputs never launch
    assert L.validate_utf8(None, 0, None).status == G.OK
    assert L.validate_utf16le(None, 0, None).status == G.OK
    assert L.utf16_length_from_utf8(None, 0, None) == 0
    assert L.utf8_length_from_utf16le(None, 0, None) == 0
    r = L.convert_utf8_to_utf16le(None, 0, None, 0, None)
    assert (r.status, r.count) == (G.OK, 0)
    # argument checks come before any device work
    assert L.validate_utf8(None, 3, None).status == G.ERR_NULL
    assert L.validate_utf16le(3, 3, None).status == G.ERR_ALIGN
    assert L.convert_utf8_to_utf16le(16, 3, 17, 3, None).status == G.ERR_ALIGN
    assert L.convert_utf8_to_utf16le(16, 3, None, 3, None).status == G.ERR_NULL
    assert L.validate_utf8(16, 1 << 40, None).status == G.ERR_TOO_BIG
    assert L.validate_utf16le(16, 1 << 38, None).status == G.ERR_TOO_BIG
    assert L.utf16_length_from_utf8(None, 3, None) == (1 << 64) - 1


def test_binding_refuses_host_tensors(G):
    import torch
    with pytest.raises(ValueError):
        G.validate_utf8(torch.zeros(4, dtype=torch.uint8))
