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


def test_read_stream_rejects_bad_arguments(lib):
    """The diagnostic read stream refuses a null context before touching a
    device (its other checks need a context, see the GPU tests)."""
    fn = lib.ch_diag_read_stream
    fn.restype, fn.argtypes = _capi.SIGNATURES["ch_diag_read_stream"]
    assert fn(None, None, 16, 0, None) == _capi.CH_E_INVALID_ARG


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


def test_serve_admission_limits(lib):
    """ch_serve_max_request_points is pure host arithmetic over the slot
    layout: it grows with the arena, shrinks with more streams, and rejects
    configurations outside the documented ranges."""
    f = lib.ch_serve_max_request_points
    f.restype = ctypes.c_uint64
    f.argtypes = [ctypes.POINTER(_capi.ServeConfig)]

    def m(arena, streams, cap=0):
        return f(ctypes.byref(_capi.ServeConfig(256, arena, 0, streams, cap)))

    assert m(64 << 30, 4) > m(8 << 30, 4) > m(1 << 30, 4) > 0
    assert m(8 << 30, 1) > m(8 << 30, 8)
    assert m(1 << 30, 0) == m(1 << 30, 4)  # 0 streams means the default 4
    assert m(1 << 30, 17) == 0 and m(1 << 30, -1) == 0
    assert m(4096, 1) == 0  # too small for any request
    # the batch cap limits what several requests share, not one request
    assert m(8 << 30, 2, 12345) == m(8 << 30, 2)
    # 10^7-point requests (the largest in the serving trace) fit a 16 GB slot.
    assert m(64 << 30, 4) >= 10**7


def test_serve_null_arguments(lib):
    lib.ch_serve_start.restype = ctypes.c_int
    lib.ch_serve_submit.restype = ctypes.c_int
    lib.ch_serve_stats.restype = ctypes.c_int
    lib.ch_serve_stop.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.ch_serve_start(None, None, ctypes.byref(out)) == 1
    t = ctypes.c_uint64()
    assert lib.ch_serve_submit(None, None, 0, ctypes.byref(t)) == 1
    assert lib.ch_serve_stats(None, None, None, None, None, None) == 1
    assert lib.ch_serve_stop(None) == 1


def test_noalloc_scratch_is_the_filter_workspace_at_its_limit(lib):
    """ch_filter_noalloc's fixed scratch is exactly ch_filter's workspace for
    CH_FILTER_NOALLOC_MAX_POINTS points, and modest (under 32 MiB)."""
    sb = lib.ch_filter_noalloc_scratch_bytes
    sb.restype = ctypes.c_size_t
    sb.argtypes = []
    f = lib.ch_filter_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_uint32]
    assert sb() == f(_capi.CH_FILTER_NOALLOC_MAX_POINTS)
    assert sb() < 32 << 20
    text = open(HEADER).read()
    assert f"#define CH_FILTER_NOALLOC_MAX_POINTS (1u << {_capi.CH_FILTER_NOALLOC_MAX_POINTS.bit_length() - 1})" in text


def test_noalloc_rejects_null_context(lib):
    fn = lib.ch_filter_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32] + [ctypes.c_void_p] * 5
    assert fn(None, None, 0, None, None, None, None, None) == _capi.CH_E_INVALID_ARG
