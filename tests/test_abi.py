"""CPU checks of the C ABI: the library loads, exports every function that
include/cga.h declares, and rejects invalid arguments on the host before any
device work is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cga.h")
LIB = os.path.join(ROOT, "paper_2110_11616_amd", "libcga.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(cga_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libcga.so not built")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


class Grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("scale", ctypes.c_float),
                ("depth", ctypes.c_uint32), ("key_mode", ctypes.c_uint32)]


def grid(depth=10, mode=0, scale=1.0):
    g = Grid()
    g.scale = scale
    g.depth = depth
    g.key_mode = mode
    return g


def test_key_widths_and_workspace_queries(lib):
    lib.cga_key_bytes.restype = ctypes.c_size_t
    lib.cga_key2_bytes.restype = ctypes.c_size_t
    for depth, kb, k2 in ((1, 4, 4), (10, 4, 4), (11, 8, 4), (16, 8, 4), (17, 8, 8), (21, 8, 8)):
        g = grid(depth)
        assert lib.cga_key_bytes(ctypes.byref(g)) == kb
        assert lib.cga_key2_bytes(ctypes.byref(g)) == k2
    for bad in (grid(0), grid(22), grid(10, 2), grid(10, 0, 0.0), grid(10, 0, float("nan"))):
        assert lib.cga_key_bytes(ctypes.byref(bad)) == 0
    for fn in ("cga_build_workspace_bytes", "cga_sort_workspace_bytes",
               "cga_project_workspace_bytes", "cga_to_arrays_workspace_bytes"):
        f = getattr(lib, fn)
        f.restype = ctypes.c_size_t
        f.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        g = grid(12)
        small, big = f(ctypes.byref(g), 1000), f(ctypes.byref(g), 10 ** 7)
        assert 256 <= small < big
        assert f(ctypes.byref(g), -1) == 0
    lib.cga_merge_workspace_bytes.restype = ctypes.c_size_t
    lib.cga_merge_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
    assert lib.cga_merge_workspace_bytes(ctypes.byref(grid(12)), 10, 10) >= 256


def test_batch_sort_bits(lib):
    """The batched sort covers the 3 * depth key bits when it is segmented
    by frame (up to 4096 frames), the frame bits too beyond that."""
    f = lib.cga_batch_sort_bits
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int]
    g = grid(12)
    assert f(ctypes.byref(g), 1) == 36
    assert f(ctypes.byref(g), 256) == 36
    assert f(ctypes.byref(g), 4096) == 36
    assert f(ctypes.byref(g), 4097) == 36 + 13
    assert f(ctypes.byref(g), 65536) == 36 + 16
    assert f(ctypes.byref(g), 0) == 0 and f(ctypes.byref(g), 65537) == 0
    assert f(ctypes.byref(grid(0)), 4) == 0


class IndexParams(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_uint32), ("leaf_kind", ctypes.c_uint32),
                ("epochs", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("root_segments", ctypes.c_uint32)]


def test_index_size_limits(lib):
    """Leaf counts 1 .. 2^24 and root segments 0 .. 65536 are accepted; the
    index grows by one 64-byte record per linear leaf and one 256-byte
    record per network leaf."""
    lib.cga_index_bytes.restype = ctypes.c_size_t
    lib.cga_index_train_workspace_bytes.restype = ctypes.c_size_t
    lib.cga_index_train_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    nb = lambda *a: lib.cga_index_bytes(ctypes.byref(IndexParams(*a)))
    for leaves in (1, 4096, 65536, 65537, 1 << 20, 1 << 24):
        for kind, rec in ((0, 64), (1, 256)):
            assert nb(leaves, kind, 50, 1e-4, 4096) >= leaves * rec
    assert nb(1 << 20, 0, 0, 0.0, 0) - nb(1 << 19, 0, 0, 0.0, 0) == (1 << 19) * 64
    for bad in ((0, 0, 0, 0.0, 0), ((1 << 24) + 1, 0, 0, 0.0, 0), (16, 2, 0, 0.0, 0),
                (16, 0, 0, 0.0, 65537)):
        assert nb(*bad) == 0
    ws = lambda leaves, n: lib.cga_index_train_workspace_bytes(
        ctypes.byref(IndexParams(leaves, 0, 0, 0.0, 0)), n)
    assert ws(1 << 24, 10) > ws(4096, 10) > 0
    assert ws((1 << 24) + 1, 10) == 0 and ws(16, -1) == 0


def test_host_validation_before_any_launch(lib):
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.cga_build.argtypes = [P, P, I64, P, P, I64, P, P, P, ctypes.c_size_t, P, P]
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    EINVAL, EWORKSPACE, EMISMATCH, EUNSUPPORTED = -1, -6, -3, -7
    g = grid(10)
    assert lib.cga_build(ctypes.byref(grid(0)), fake, 10, fake, None, 10, None, None, fake, 1 << 30,
                         None, None) == EINVAL
    assert lib.cga_build(ctypes.byref(g), fake, -1, fake, None, 10, None, None, fake, 1 << 30,
                         None, None) == EINVAL
    assert lib.cga_build(ctypes.byref(g), None, 10, fake, None, 10, None, None, fake, 1 << 30,
                         None, None) == EINVAL
    assert lib.cga_build(ctypes.byref(g), fake, 10, fake, None, 10, None, None, fake, 16,
                         None, None) == EWORKSPACE
    assert lib.cga_build(ctypes.byref(g), fake, 1 << 30, fake, None, 10, None, None, fake, 1 << 40,
                         None, None) == EUNSUPPORTED
    lib.cga_knn.argtypes = [P, P, I64, P, P, I64, ctypes.c_int, P, P, P, ctypes.c_size_t, P]
    for k in (0, 33):
        assert lib.cga_knn(ctypes.byref(g), fake, 10, None, fake, 5, k, fake, fake, fake, 256,
                           None) == EINVAL
    # LINEAR grids are searched too (through a Morton re-key), so the tiny
    # workspace is what fails
    assert lib.cga_knn(ctypes.byref(grid(10, 1)), fake, 10, None, fake, 5, 1, fake, fake, fake, 256,
                       None) == EWORKSPACE
    assert lib.cga_knn(ctypes.byref(g), fake, 1 << 31, None, fake, 5, 1, fake, fake, fake, 256,
                       None) == EINVAL
    lib.cga_project.argtypes = [P, P, I64, P, ctypes.c_int, P, P, I64, P, P, P, ctypes.c_size_t,
                                P, P]
    for axis in (-1, 3):
        assert lib.cga_project(ctypes.byref(g), fake, 10, None, axis, fake, None, 10, None, None,
                               fake, 1 << 30, None, None) == EINVAL
    lib.cga_to_arrays.argtypes = [P, P, I64, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]
    assert lib.cga_to_arrays(ctypes.byref(grid(10, 0)), fake, 10, None, fake, fake, fake, fake,
                             fake, None, None, None, None, fake, 1 << 30, None) == EMISMATCH
    lib.cga_strerror.restype = ctypes.c_char_p
    assert lib.cga_strerror(-4) == b"non-finite coordinate"


def test_merge_noalloc_rejects_sizes_beyond_its_static_scratch(lib):
    """cga_merge_noalloc (no workspace argument) refuses more than
    CGA_MERGE_NOALLOC_MAX_KEYS merged positions, and bad arguments, on the
    host, before it touches the device."""
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.cga_merge_noalloc.argtypes = [P, P, I64, P, P, I64, P, P, P, I64, P, P, P]
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    EINVAL, EWORKSPACE = -1, -6
    text = open(HEADER).read()
    cap = int(re.search(r"CGA_MERGE_NOALLOC_MAX_KEYS \(\(int64_t\)1 << (\d+)\)", text).group(1))
    mx = 1 << cap
    g = grid(12)
    call = lambda na, nb, gg=g, a=fake, out=fake: lib.cga_merge_noalloc(
        ctypes.byref(gg), a, na, None, fake, nb, None, out, None, min(max(na + nb, 0), 1 << 62),
        None, None, None)
    assert call(mx, 1) == EWORKSPACE
    assert call(1, mx) == EWORKSPACE
    assert call(mx // 2 + 1, mx // 2) == EWORKSPACE
    assert call(1 << 62, 1 << 62) == EWORKSPACE
    assert call(-1, 5) == EINVAL
    assert call(5, 5, gg=grid(0)) == EINVAL
    assert call(5, 5, a=None) == EINVAL
    assert call(5, 5, out=None) == EINVAL
