"""Host-side checks of the C ABI (no GPU needed, no kernel launched)."""
import ctypes
import os
import re

import pytest

from paper_2209_12310_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "convhull.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ch_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_capi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(_capi.LIB_PATH)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "ch_filter" in names and "ch_hull" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_declares_exactly_the_header(lib):
    assert sorted(_capi.SIGNATURES) == _declared()


def test_status_strings(lib):
    lib.ch_status_string.restype = ctypes.c_char_p
    assert lib.ch_status_string(0) == b"ok"
    assert b"grid" in lib.ch_status_string(2)
    assert lib.ch_status_string(99) == b"unknown status"


def test_workspace_sizes(lib):
    f = lib.ch_filter_workspace_bytes
    h = lib.ch_hull_workspace_bytes
    f.restype = h.restype = ctypes.c_size_t
    f.argtypes = h.argtypes = [ctypes.c_uint32]
    prev = 0
    for n in [0, 1, 2, 255, 4096, 4097, 10**6, 10**8, 2**31 - 1]:
        assert f(n) % 256 == 0 and h(n) % 256 == 0
        assert h(n) >= f(n) >= prev
        prev = f(n)
    assert h(10**8) < 64 * 10**8  # bounded per point


def test_null_context_is_rejected(lib):
    lib.ch_filter.restype = ctypes.c_int
    assert lib.ch_filter(None, None, 0, None, None, None, None, None, 0, None) == 1


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2209_12310_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "oracle.c" not in text and "liboracle" not in text, fn
    text = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert "convhull.h" not in text and "ch_internal" not in text


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    import paper_2209_12310_amd as ch
    with pytest.raises(TypeError):
        ch._check_points(torch.zeros((4, 2), dtype=torch.float32))
