"""GPU parity: every entry point of the HIP library against the CPU oracle,
bit-exact, on seeded workloads sized to span several tiles with ragged tails,
plus the edge cases (empty, single, all-equal, depth limits, non-finite,
capacity, padding)."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gen import Grid
from helpers import dev, keys_dev, say, u32, u64

pytestmark = pytest.mark.gpu
M, L = gen.KEY_MORTON, gen.KEY_LINEAR


@pytest.fixture(scope="module")
def w_c1():
    return gen.c1_spheres()


@pytest.fixture(scope="module")
def w_c2s():
    # the LiDAR workload at 1/16 of the azimuth steps (65,536 points per sweep)
    return gen.c2_lidar(naz=1024, nq=20000)


@pytest.fixture(scope="module")
def w_c3s():
    return gen.c3_bumpy(n=300_000, nq=20000)


def _wl(name, request):
    return request.getfixturevalue(name)


# ------------------------------------------------------------------ encode
@pytest.mark.parametrize("wl", ["w_c1", "w_c2s", "w_c3s"])
@pytest.mark.parametrize("mode", [M, L])
def test_encode(gpu, wl, mode, request):
    d = _wl(wl, request)
    g = d["grid"].with_mode(mode)
    say("encode", wl, mode)
    k = gpu.cga_encode_keys(dev(d["a"]), g)
    want = oracle.encode(oracle.quantize(d["a"], g), g.depth, mode)
    assert np.array_equal(u64(k), want)


def test_encode_edges(gpu):
    g = Grid((0.0, 0.0, 0.0), 1024.0, 10, M)
    p = np.array([[1 - 2 ** -24, 0.0, 0.5], [-1e-7, 1.0, 5.0], [-3.0, 1e30, -1e30],
                  [0.25, 0.5, 0.75]], np.float32)
    k = gpu.cga_encode_keys(dev(p), g)
    assert np.array_equal(u64(k), oracle.encode(oracle.quantize(p, g), 10, M))
    g2 = Grid((2.0 ** -25, 0.0, 0.0), 512.0, 10, L)  # rounding of the subtract decides
    k = gpu.cga_encode_keys(dev(np.array([[1.0, 0.0, 0.0]], np.float32)), g2)
    assert int(u64(k)[0]) >> 20 == 512


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite(gpu, bad):
    g = Grid((0.0, 0.0, 0.0), 16.0, 4, M)
    p = np.random.default_rng(0).uniform(0, 1, (5000, 3)).astype(np.float32)
    p[1234, 1] = bad
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_build(dev(p), g)
    assert e.value.status == gpu.ENONFINITE
    with pytest.raises(gpu.CgaError):
        gpu.cga_knn(keys_dev(np.array([1, 2], np.uint64), g), dev(p[1230:1240]), g, 1)


# -------------------------------------------------------------------- sort
@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 4097, 3 * 3072 + 5, 300_001])
@pytest.mark.parametrize("depth,bits", [(10, 30), (12, 36), (16, 48), (21, 63)])
def test_sort(gpu, n, depth, bits):
    rng = np.random.default_rng(n + bits)
    keys = rng.integers(0, 2 ** bits, n, dtype=np.uint64)
    keys[: n // 3] = keys[0]  # many equal keys
    g = Grid((0.0, 0.0, 0.0), 1.0, depth, M)
    say("sort", n, bits)
    out = gpu.cga_sort_keys(keys_dev(keys, g), g)
    assert np.array_equal(u64(out), np.sort(keys))


@pytest.mark.parametrize("rb", [4, 5, 6, 7, 8, 9, 10, 11])
@pytest.mark.parametrize("items", [8, 12, 16, 24, 32])
def test_sort_every_tuning(gpu, rb, items):
    rng = np.random.default_rng(rb * 100 + items)
    keys = rng.integers(0, 2 ** 44, 70_001, dtype=np.uint64)
    keys[::7] = keys[3]
    g = Grid((0.0, 0.0, 0.0), 1.0, 15, M)
    out = gpu.cga_sort_keys(keys_dev(keys, g), g, key_bits=45, tune=(rb, items))
    assert np.array_equal(u64(out), np.sort(keys))
    g32 = Grid((0.0, 0.0, 0.0), 1.0, 10, M)
    k32 = (keys & np.uint64(2 ** 30 - 1))
    out = gpu.cga_sort_keys(keys_dev(k32, g32), g32, tune=(rb, items))
    assert np.array_equal(u64(out), np.sort(k32))


# ------------------------------------------------------------------- build
def _check_build(gpu, xyz, g, tune=None):
    k, c = gpu.cga_build(dev(xyz), g, tune=tune)
    wk, wc = oracle.build(xyz, g)
    assert np.array_equal(u64(k), wk)
    assert np.array_equal(u32(c), wc)
    return wk


@pytest.mark.parametrize("wl", ["w_c1", "w_c2s", "w_c3s"])
@pytest.mark.parametrize("mode", [M, L])
def test_build(gpu, wl, mode, request):
    d = _wl(wl, request)
    say("build", wl, mode)
    _check_build(gpu, d["a"], d["grid"].with_mode(mode))


@pytest.mark.parametrize("tune", [(4, 8), (6, 12), (9, 16), (11, 8)])
def test_build_tunings_identical(gpu, w_c2s, tune):
    _check_build(gpu, w_c2s["a"], w_c2s["grid"], tune)


@pytest.mark.parametrize("depth", [1, 2, 10, 11, 16, 21])
def test_build_depths(gpu, depth):
    rng = np.random.default_rng(depth)
    xyz = rng.uniform(-0.1, 1.1, (50_000, 3)).astype(np.float32)
    g = Grid((0.0, 0.0, 0.0), float(np.float32(2.0 ** depth)), depth, M)
    for mode in (M, L):
        _check_build(gpu, xyz, g.with_mode(mode))


@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097])
def test_build_sizes_and_duplicates(gpu, n):
    g = Grid((0.0, 0.0, 0.0), 1.0, 6, M)
    rng = np.random.default_rng(n)
    _check_build(gpu, rng.integers(0, 64, (n, 3)).astype(np.float32), g)
    same = np.tile(np.array([[5.0, 9.0, 33.0]], np.float32), (max(n, 1), 1))
    k, c = gpu.cga_build(dev(same), g)
    assert len(k) == 1 and int(u32(c)[0]) == len(same)


def test_build_capacity(gpu, w_c1):
    g = w_c1["grid"]
    _, wc = oracle.build(w_c1["a"], g)
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_build(dev(w_c1["a"]), g, cap=len(wc) - 1)
    assert e.value.status == gpu.ECAPACITY
    k, _ = gpu.cga_build(dev(w_c1["a"]), g, cap=len(wc))
    assert len(k) == len(wc)


# ------------------------------------------------------------ paper arrays
@pytest.mark.parametrize("wl", ["w_c1", "w_c2s"])
def test_to_arrays(gpu, wl, request):
    d = _wl(wl, request)
    g = d["grid"].with_mode(L)
    k, _ = gpu.cga_build(dev(d["a"]), g)
    arr = gpu.cga_to_arrays(k, g)
    want = oracle.arrays(u64(k), g.depth, L)
    for name in ("x_index", "y_index", "z_index"):
        assert np.array_equal(u32(arr[name]), want[name]), name
    for name in ("x_pointer", "y_pointer"):
        assert np.array_equal(arr[name].cpu().numpy(), want[name]), name


def test_to_arrays_table2(gpu):
    import json
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden")
    pts = np.array(json.load(open(os.path.join(gold, "table2_points.json")))["soldier"], np.float32)
    want = json.load(open(os.path.join(gold, "table2_derived.json")))["soldier_arrays"]
    g = Grid((0.0, 0.0, 0.0), 1.0, 8, L)
    k, _ = gpu.cga_build(dev(pts), g)
    arr = gpu.cga_to_arrays(k, g)
    for name, v in want.items():
        got = arr[name].cpu().numpy()
        got = got.view(np.uint32) if got.dtype == np.int32 else got
        assert got.tolist() == v, name


# ------------------------------------------- the paper's array operations
def _lin_arrays(gpu, xyz, g):
    k, _ = gpu.cga_build(dev(xyz), g)
    return k, gpu.cga_to_arrays(k, g), oracle.arrays(u64(k), g.depth, L)


@pytest.mark.parametrize("wl", ["w_c1", "w_c2s", "w_c3s"])
def test_arrays_lookup(gpu, wl, request):
    d = _wl(wl, request)
    g = d["grid"].with_mode(L)
    k, arr, oarr = _lin_arrays(gpu, d["a"], g)
    keys = u64(k)
    rng = np.random.default_rng(71)
    top = 2 ** g.depth
    qv = np.concatenate([oracle.decode(keys[rng.integers(0, len(keys), 20000)], g.depth, L),
                         rng.integers(0, top, (20000, 3)),
                         [[0, 0, 0], [top - 1] * 3, [top, 0, 0], [2 ** 32 - 1] * 3]]).astype(np.uint32)
    say("arrays lookup", wl, len(keys), len(qv))
    pos = gpu.cga_arrays_lookup(arr, dev(qv.view(np.int32)), g).cpu().numpy()
    want = oracle.lookup_cga(oarr, qv)
    np.testing.assert_array_equal(pos, want)
    assert (pos[:20000] >= 0).all()
    ok = qv.max(1) < top  # membership and rank in the key array say the same
    rank, found = oracle.lower_bound(keys, oracle.encode(qv[ok], g.depth, L))
    np.testing.assert_array_equal(pos[ok], np.where(found.astype(bool), rank, -1))


@pytest.mark.parametrize("wl", ["w_c1", "w_c2s", "w_c3s"])
def test_arrays_nn(gpu, wl, request):
    d = _wl(wl, request)
    g = d["grid"].with_mode(L)
    k, arr, oarr = _lin_arrays(gpu, d["a"], g)
    q = d["q"]
    say("arrays nn", wl, len(k), len(q))
    idx, d2 = gpu.cga_arrays_nn(arr, dev(q), g)
    idx, d2 = idx.cpu().numpy(), d2.cpu().numpy().view(np.uint64)
    widx, wd2 = oracle.knn_kdtree(u64(k), q, g, 1)  # same order: (distance, LINEAR key)
    np.testing.assert_array_equal(d2, wd2[:, 0])
    np.testing.assert_array_equal(idx, widx[:, 0])
    rows = np.arange(0, len(q), max(1, len(q) // 300))  # the paper's own steps, on a sample
    qv = oracle.quantize(q[rows], g).astype(np.uint32)
    ppos, pd2 = oracle.nn_cga(oarr, qv, g.depth, L)
    np.testing.assert_array_equal(idx[rows], ppos)
    np.testing.assert_array_equal(d2[rows], pd2)


def test_arrays_edges(gpu):
    rng = np.random.default_rng(73)
    g = Grid((0.0, 0.0, 0.0), 1.0, 5, L)  # tiny grid: many exact ties
    pts = rng.integers(0, 32, (300, 3)).astype(np.float32)
    k, arr, oarr = _lin_arrays(gpu, pts, g)
    q = np.concatenate([pts[:50], rng.integers(-3, 35, (400, 3)).astype(np.float32)])
    idx, d2 = gpu.cga_arrays_nn(arr, dev(q), g)
    widx, wd2 = oracle.knn_brute(u64(k), q, g, 1)
    np.testing.assert_array_equal(d2.cpu().numpy().view(np.uint64), wd2[:, 0])
    np.testing.assert_array_equal(idx.cpu().numpy(), widx[:, 0])
    for m in (1, 2):  # one voxel; two voxels
        km, am, _ = _lin_arrays(gpu, pts[:m], g)
        idx, d2 = gpu.cga_arrays_nn(am, dev(q), g)
        widx, wd2 = oracle.knn_brute(u64(km), q, g, 1)
        np.testing.assert_array_equal(idx.cpu().numpy(), widx[:, 0])
        np.testing.assert_array_equal(d2.cpu().numpy().view(np.uint64), wd2[:, 0])
    empty = gpu.cga_to_arrays(k[:0], g)
    idx, d2 = gpu.cga_arrays_nn(empty, dev(q[:5]), g)
    assert (idx.cpu().numpy() == -1).all() and (d2.cpu().numpy() == -1).all()
    assert (gpu.cga_arrays_lookup(empty, dev(np.zeros((3, 3), np.int32)), g).cpu().numpy() == -1).all()
    bad = q[:10].copy()
    bad[4, 1] = np.inf
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_arrays_nn(arr, dev(bad), g)
    assert e.value.status == gpu.ENONFINITE
    with pytest.raises(gpu.CgaError) as e:  # MORTON grids have no such arrays
        gpu.cga_arrays_nn(arr, dev(q[:3]), g.with_mode(M))
    assert e.value.status == gpu.EMISMATCH
    # a pointer past the end of Y_index: flagged, every access clamped in bounds
    broken = dict(arr)
    xp = arr["x_pointer"].clone()
    xp[1:-1] = xp[-1] + 1000
    broken["x_pointer"] = xp
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_arrays_nn(broken, dev(q), g)
    assert e.value.status == gpu.EMISMATCH


# ------------------------------------------------------------------- merge
@pytest.mark.parametrize("wl", ["w_c1", "w_c2s", "w_c3s"])
@pytest.mark.parametrize("mode", [M, L])
def test_merge(gpu, wl, mode, request):
    d = _wl(wl, request)
    g = d["grid"].with_mode(mode)
    ka, _ = gpu.cga_build(dev(d["a"]), g)
    kb, _ = gpu.cga_build(dev(d["b"]), g)
    say("merge", wl, mode, len(ka), len(kb))
    m, s = gpu.cga_merge(ka, kb, g, src=True)
    wm, ws = oracle.merge(u64(ka), u64(kb), g.depth, mode)
    assert np.array_equal(u64(m), wm)
    assert np.array_equal(s.cpu().numpy(), ws)


def test_merge_edges(gpu):
    g = Grid((0.0, 0.0, 0.0), 1.0, 12, M)
    rng = np.random.default_rng(9)
    a = np.unique(rng.integers(0, 2 ** 36, 20_000, dtype=np.uint64))
    b = np.unique(np.concatenate([a[::3], rng.integers(0, 2 ** 36, 9_000, dtype=np.uint64)]))
    cases = [(a, b), (b, a), (a, a), (a, a[:0]), (a[:0], b), (a[:0], a[:0]), (a[:1], a[1:2]),
             (a[:2048], a[2048:4096]), (a[::2], a[1::2])]
    for x, y in cases:
        m, s = gpu.cga_merge(keys_dev(x, g), keys_dev(y, g), g, src=True)
        wm, ws = oracle.merge(x, y, 12, M)
        assert np.array_equal(u64(m), wm)
        assert np.array_equal(s.cpu().numpy(), ws)
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_merge(keys_dev(a, g), keys_dev(b, g), g, cap=len(np.union1d(a, b)) - 1)
    assert e.value.status == gpu.ECAPACITY


# -------------------------------------------------------------- projection
@pytest.mark.parametrize("wl", ["w_c1", "w_c2s", "w_c3s"])
@pytest.mark.parametrize("mode", [M, L])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_project(gpu, wl, mode, axis, request):
    d = _wl(wl, request)
    g = d["grid"].with_mode(mode)
    k, _ = gpu.cga_build(dev(d["a"]), g)
    say("project", wl, mode, axis)
    p, c = gpu.cga_project(k, g, axis)
    wp, wc = oracle.project(u64(k), g.depth, mode, axis)
    assert np.array_equal(u64(p), wp)
    assert np.array_equal(u32(c), wc)


def test_project_depth_limits(gpu):
    rng = np.random.default_rng(17)
    for depth in (16, 17, 21):  # 2-D keys switch to 64 bits above depth 16
        g = Grid((0.0, 0.0, 0.0), float(2 ** depth), depth, M)
        xyz = rng.uniform(0, 1, (40_000, 3)).astype(np.float32)
        for mode in (M, L):
            gm = g.with_mode(mode)
            k, _ = gpu.cga_build(dev(xyz), gm)
            for axis in (0, 1, 2):
                p, c = gpu.cga_project(k, gm, axis)
                wp, wc = oracle.project(u64(k), depth, mode, axis)
                assert np.array_equal(u64(p), wp) and np.array_equal(u32(c), wc)


# --------------------------------------------------------------------- kNN
def _check_knn(gpu, keys_gpu, q, g, k, tier="kd"):
    idx, d2 = gpu.cga_knn(keys_gpu, dev(q), g, k)
    keys = u64(keys_gpu)
    fn = oracle.knn_kdtree if tier == "kd" else oracle.knn_brute
    widx, wd2 = fn(keys, q, g, k)
    assert np.array_equal(d2.cpu().numpy().view(np.uint64), wd2)
    assert np.array_equal(idx.cpu().numpy(), widx)


def test_knn_c1(gpu, w_c1):
    g = w_c1["grid"]
    ka, _ = gpu.cga_build(dev(w_c1["a"]), g)
    kb, _ = gpu.cga_build(dev(w_c1["b"]), g)
    m, _ = gpu.cga_merge(ka, kb, g)
    _check_knn(gpu, m, w_c1["q"], g, 1, tier="brute")


@pytest.mark.parametrize("k", [1, 3, 8, 16, 32])
def test_knn_c2s(gpu, w_c2s, k):
    g = w_c2s["grid"]
    ka, _ = gpu.cga_build(dev(w_c2s["a"]), g)
    say("knn c2s", k)
    _check_knn(gpu, ka, w_c2s["q"], g, k)


@pytest.mark.parametrize("k", [1, 16])
def test_knn_c3s(gpu, w_c3s, k):
    g = w_c3s["grid"]
    ka, _ = gpu.cga_build(dev(w_c3s["a"]), g)
    _check_knn(gpu, ka, w_c3s["q"], g, k)


def test_knn_edges(gpu):
    rng = np.random.default_rng(21)
    g = Grid((0.0, 0.0, 0.0), 1.0, 5, M)  # tiny grid: many exact ties
    pts = rng.integers(0, 32, (300, 3)).astype(np.float32)
    k_, _ = gpu.cga_build(dev(pts), g)
    q = np.concatenate([pts[:50], rng.integers(-3, 35, (200, 3)).astype(np.float32)])
    for k in (1, 2, 5, 8, 13, 32):
        _check_knn(gpu, k_, q, g, k, tier="brute")
    few = k_[:3]  # fewer voxels than k: padding
    _check_knn(gpu, few, q[:20], g, 8, tier="brute")
    empty = k_[:0]
    idx, d2 = gpu.cga_knn(empty, dev(q[:4]), g, 2)
    assert (idx.cpu().numpy() == -1).all()
    g21 = Grid((0.0, 0.0, 0.0), float(2 ** 21), 21, M)
    xyz = rng.uniform(0, 1, (20_000, 3)).astype(np.float32)
    k21, _ = gpu.cga_build(dev(xyz), g21)
    _check_knn(gpu, k21, rng.uniform(0, 1, (500, 3)).astype(np.float32), g21, 4)


@pytest.mark.parametrize("k", [1, 8, 16])
def test_knn_query_order(gpu, w_c2s, monkeypatch, k):
    """The Morton ordering of the queries (on by default from 2^18 queries,
    forced here at small sizes) leaves every row where it belongs."""
    monkeypatch.setenv("CGA_KNN_ORDER", "1")
    g = w_c2s["grid"]
    ka, _ = gpu.cga_build(dev(w_c2s["a"]), g)
    say("knn ordered c2s", k)
    _check_knn(gpu, ka, w_c2s["q"], g, k)
    rng = np.random.default_rng(23)
    g5 = Grid((0.0, 0.0, 0.0), 1.0, 5, M)  # ties; a ragged query count
    pts = rng.integers(0, 32, (300, 3)).astype(np.float32)
    k5, _ = gpu.cga_build(dev(pts), g5)
    q = rng.integers(-3, 35, (4097, 3)).astype(np.float32)
    _check_knn(gpu, k5, q, g5, k, tier="brute")
    _check_knn(gpu, k5, q[:1], g5, k, tier="brute")
    g21 = Grid((0.0, 0.0, 0.0), float(2 ** 21), 21, M)  # key bits beyond the ordering's 24
    k21, _ = gpu.cga_build(dev(rng.uniform(0, 1, (20_000, 3)).astype(np.float32)), g21)
    _check_knn(gpu, k21, rng.uniform(0, 1, (3000, 3)).astype(np.float32), g21, k)
    bad = q[:100].copy()
    bad[57, 2] = np.nan
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_knn(k5, dev(bad), g5, k)
    assert e.value.status == gpu.ENONFINITE


@pytest.mark.parametrize("k", [1, 8, 16, 32])
@pytest.mark.parametrize("ordered", ["0", "1"])
def test_knn_query_queue(gpu, w_c2s, monkeypatch, k, ordered):
    """Teams taking their queries from the counter (on by default from 8
    queries per resident team, forced here at small sizes, with and without
    the Morton ordering) leave every row where it belongs: ties, a ragged
    query count, wide lists, a non-finite query, and the counting build."""
    monkeypatch.setenv("CGA_KNN_QUEUE", "1")
    monkeypatch.setenv("CGA_KNN_ORDER", ordered)
    g = w_c2s["grid"]
    ka, _ = gpu.cga_build(dev(w_c2s["a"]), g)
    say("knn queue c2s", k, ordered)
    _check_knn(gpu, ka, w_c2s["q"], g, k)
    idx, d2, work = gpu.cga_knn_count(ka, dev(w_c2s["q"]), g, k)
    widx, wd2 = oracle.knn_kdtree(u64(ka), w_c2s["q"], g, k)
    np.testing.assert_array_equal(d2.cpu().numpy().view(np.uint64), wd2)
    np.testing.assert_array_equal(idx.cpu().numpy(), widx)
    assert work["node_loads"] > 0 and work["steps"] > 0
    rng = np.random.default_rng(31)
    g5 = Grid((0.0, 0.0, 0.0), 1.0, 5, M)
    pts = rng.integers(0, 32, (300, 3)).astype(np.float32)
    k5, _ = gpu.cga_build(dev(pts), g5)
    q = rng.integers(-3, 35, (4097, 3)).astype(np.float32)
    _check_knn(gpu, k5, q, g5, k, tier="brute")
    _check_knn(gpu, k5, q[:1], g5, k, tier="brute")
    g21 = Grid((0.0, 0.0, 0.0), float(2 ** 21), 21, M)
    k21, _ = gpu.cga_build(dev(rng.uniform(0, 1, (20_000, 3)).astype(np.float32)), g21)
    _check_knn(gpu, k21, rng.uniform(0, 1, (3000, 3)).astype(np.float32), g21, k)
    bad = q[:100].copy()
    bad[57, 2] = np.nan
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_knn(k5, dev(bad), g5, k)
    assert e.value.status == gpu.ENONFINITE


@pytest.mark.parametrize("k", [1, 8, 16, 32])
@pytest.mark.parametrize("queue", ["0", "1"])
@pytest.mark.parametrize("blocks", ["1", "3"])
def test_knn_few_blocks(gpu, w_c2s, monkeypatch, k, queue, blocks):
    """A grid of one or three blocks (32 or 96 teams of 8 lanes, 16 or 48 of
    16) answers every query: each team goes through many queries in turn,
    from the counter or round-robin, with ties, a ragged count, wide lists
    and a non-finite query among them."""
    monkeypatch.setenv("CGA_KNN_BLOCKS", blocks)
    monkeypatch.setenv("CGA_KNN_QUEUE", queue)
    g = w_c2s["grid"]
    ka, _ = gpu.cga_build(dev(w_c2s["a"]), g)
    say("knn few blocks c2s", k, queue, blocks)
    q = w_c2s["q"][:20_000]
    _check_knn(gpu, ka, q, g, k)
    rng = np.random.default_rng(37)
    g5 = Grid((0.0, 0.0, 0.0), 1.0, 5, M)
    pts = rng.integers(0, 32, (300, 3)).astype(np.float32)
    k5, _ = gpu.cga_build(dev(pts), g5)
    q5 = rng.integers(-3, 35, (3001, 3)).astype(np.float32)
    _check_knn(gpu, k5, q5, g5, k, tier="brute")
    g21 = Grid((0.0, 0.0, 0.0), float(2 ** 21), 21, M)
    k21, _ = gpu.cga_build(dev(rng.uniform(0, 1, (20_000, 3)).astype(np.float32)), g21)
    _check_knn(gpu, k21, rng.uniform(0, 1, (3000, 3)).astype(np.float32), g21, k)
    bad = q5[:500].copy()
    bad[333, 0] = np.inf
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_knn(k5, dev(bad), g5, k)
    assert e.value.status == gpu.ENONFINITE


def test_knn_query_order_auto(gpu, w_c2s):
    """At 2^18 queries the ordering switches on by itself; the rows equal
    those of the unordered search on the same queries."""
    g = w_c2s["grid"]
    ka, _ = gpu.cga_build(dev(w_c2s["a"]), g)
    rng = np.random.default_rng(29)
    q = w_c2s["q"][rng.integers(0, len(w_c2s["q"]), 1 << 18)]
    q = q + rng.uniform(-0.5, 0.5, q.shape).astype(np.float32)
    idx, d2 = gpu.cga_knn(ka, dev(q), g, 4)
    rows = np.sort(rng.choice(len(q), 3000, replace=False))
    widx, wd2 = oracle.knn_kdtree(u64(ka), q[rows], g, 4)
    np.testing.assert_array_equal(d2.cpu().numpy().view(np.uint64)[rows], wd2)
    np.testing.assert_array_equal(idx.cpu().numpy()[rows], widx)


@pytest.mark.parametrize("k", [1, 8, 16])
def test_knn_count_same_results(gpu, w_c2s, k):
    """The counting build of the search returns the rows of cga_knn (checked
    against the kd-tree) and deterministic work totals: at least one node
    load and loop step per query and at least k offered voxels per query."""
    g = w_c2s["grid"]
    ka, _ = gpu.cga_build(dev(w_c2s["a"]), g)
    q = dev(w_c2s["q"])
    idx, d2 = gpu.cga_knn(ka, q, g, k)
    ci, cd, w1 = gpu.cga_knn_count(ka, q, g, k)
    assert torch.equal(ci, idx) and torch.equal(cd, d2)
    _, _, w2 = gpu.cga_knn_count(ka, q, g, k)
    assert w1 == w2
    nq = len(w_c2s["q"])
    assert w1["node_loads"] >= nq and w1["steps"] >= nq and w1["voxels_offered"] >= k * nq
    widx, wd2 = oracle.knn_kdtree(u64(ka), w_c2s["q"], g, k)
    assert np.array_equal(ci.cpu().numpy(), widx) and np.array_equal(cd.cpu().numpy().view(np.uint64), wd2)


def test_stream_probe_copies(gpu):
    """The bandwidth probe's copy writes exactly its source; its read mode
    writes nothing."""
    n = (64 << 20) + 16 * 1001
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (n // 4,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    for blocks in (1, 977, 4096):
        dst.zero_()
        gpu.cga_stream_probe(src, dst, n, 0, blocks)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
    sink = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    gpu.cga_stream_probe(src, sink, n, 1, 4096)
    torch.cuda.synchronize()
    assert int(sink.item()) == 7 or int(sink.item()) == 0x9E3779B9 - 2 ** 32


# --------------------------------------------------------------- occupancy
def _check_occupancy(gpu, keys_gpu, g):
    codes, counts = gpu.cga_occupancy(keys_gpu, g)
    wcodes, wcounts = oracle.occupancy(u64(keys_gpu), g.depth)
    np.testing.assert_array_equal(counts.cpu().numpy(), wcounts)
    np.testing.assert_array_equal(codes.cpu().numpy(), wcodes)


@pytest.mark.parametrize("wl", ["w_c1", "w_c2s", "w_c3s"])
def test_occupancy(gpu, wl, request):
    d = _wl(wl, request)
    g = d["grid"]
    k, _ = gpu.cga_build(dev(d["a"]), g)
    say("occupancy", wl, k.shape[0])
    _check_occupancy(gpu, k, g)


@pytest.mark.parametrize("depth", [1, 2, 7, 8, 11, 21])
def test_occupancy_depths(gpu, depth):
    rng = np.random.default_rng(40 + depth)
    g = Grid((0.0, 0.0, 0.0), float(2 ** depth), depth, M)
    xyz = rng.uniform(0, 1, (3000, 3)).astype(np.float32)
    k, _ = gpu.cga_build(dev(xyz), g)
    _check_occupancy(gpu, k, g)


def test_occupancy_edges(gpu, w_c1):
    g = w_c1["grid"]
    k, _ = gpu.cga_build(dev(w_c1["a"]), g)
    _check_occupancy(gpu, k[:1], g)
    codes, counts = gpu.cga_occupancy(k[:0], g)
    assert codes.numel() == 0 and counts.cpu().numpy().tolist() == [0] * (g.depth + 1)
    # counts only (no code buffer), and a code buffer one byte short
    cnt = torch.empty(g.depth + 1, dtype=torch.int64, device="cuda")
    wcodes, wcounts = oracle.occupancy(u64(k), g.depth)
    ws = gpu.Workspaces("cuda")
    wsb = gpu._ws("occupancy", gpu.lib.cga_occupancy_workspace_bytes(
        gpu.ctypes.byref(gpu.grid_struct(g)), k.shape[0]), ws)
    assert gpu.lib.cga_occupancy(gpu.ctypes.byref(gpu.grid_struct(g)), gpu._ptr(k), k.shape[0],
                                 None, None, 0, gpu._ptr(cnt), gpu._ptr(wsb), wsb.numel(),
                                 gpu._stream()) == 0
    assert gpu.lib.cga_ws_status(gpu._ptr(wsb), gpu._stream()) == 0
    np.testing.assert_array_equal(cnt.cpu().numpy(), wcounts)
    short = torch.empty(len(wcodes) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_occupancy(k, g, occ_out=short)
    assert e.value.status == gpu.ECAPACITY
    np.testing.assert_array_equal(short.cpu().numpy(), wcodes[:-1])


def test_occupancy_linear_unsupported(gpu, w_c1):
    g = w_c1["grid"].with_mode(L)
    k, _ = gpu.cga_build(dev(w_c1["a"]), g)
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_occupancy(k, g)
    assert e.value.status == gpu.EUNSUPPORTED


# ------------------------------------------------------------------ values
def _u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("wl", ["w_c1", "w_c2s", "w_c3s"])
@pytest.mark.parametrize("mode", [M, L])
def test_voxel_values(gpu, wl, mode, request):
    d = _wl(wl, request)
    g = d["grid"].with_mode(mode)
    attr = gen.attributes(51, 1, len(d["a"]))
    k, _ = gpu.cga_build(dev(d["a"]), g)
    v = gpu.cga_voxel_values(dev(d["a"]), dev(attr.view(np.int32)), k, g)
    wk, wv = oracle.voxel_values(d["a"], attr, g)
    np.testing.assert_array_equal(u64(k), wk)
    np.testing.assert_array_equal(_u32(v), wv)


@pytest.mark.parametrize("policy", [0, 1])
@pytest.mark.parametrize("wl", ["w_c1", "w_c2s"])
def test_merge_values(gpu, wl, policy, request):
    d = _wl(wl, request)
    g = d["grid"]
    aa, ab = gen.attributes(52, 1, len(d["a"])), gen.attributes(52, 2, len(d["b"]))
    ka, _ = gpu.cga_build(dev(d["a"]), g)
    kb, _ = gpu.cga_build(dev(d["b"]), g)
    va = gpu.cga_voxel_values(dev(d["a"]), dev(aa.view(np.int32)), ka, g)
    vb = gpu.cga_voxel_values(dev(d["b"]), dev(ab.view(np.int32)), kb, g)
    km, _ = gpu.cga_merge(ka, kb, g)
    vm = gpu.cga_merge_values(ka, va, kb, vb, km, g, policy)
    wka, wva = oracle.voxel_values(d["a"], aa, g)
    wkb, wvb = oracle.voxel_values(d["b"], ab, g)
    wkm, wvm = oracle.merge_values(wka, wva, wkb, wvb, policy)
    np.testing.assert_array_equal(u64(km), wkm)
    np.testing.assert_array_equal(_u32(vm), wvm)


def test_values_edges(gpu, w_c1):
    g = w_c1["grid"]
    pts = np.zeros((5, 3), np.float32)   # all in one voxel
    attr = np.array([1, 2, 2, 2, 2], np.uint32) | (np.array([255, 255, 0, 0, 0], np.uint32) << 8)
    k, _ = gpu.cga_build(dev(pts), g)
    v = gpu.cga_voxel_values(dev(pts), dev(attr.view(np.int32)), k, g)
    assert _u32(v).tolist() == oracle.voxel_values(pts, attr, g)[1].tolist()
    # a point whose voxel is not among the keys
    other = np.ones((1, 3), np.float32) * 0.5
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_voxel_values(dev(other), dev(attr[:1].view(np.int32)), k, g)
    assert e.value.status == gpu.EMISMATCH
    # empty clouds
    ke = k[:0]
    assert gpu.cga_voxel_values(dev(pts[:0]), dev(attr[:0].view(np.int32)), ke, g).numel() == 0
    vm = gpu.cga_merge_values(k, v, ke, v[:0], k, g, 1)
    assert _u32(vm).tolist() == _u32(v).tolist()
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_merge_values(k, v, ke, v[:0], k, g, 2)
    assert e.value.status == gpu.EINVAL


def test_values_runs(gpu, w_c1):
    """Runs of equal voxels among consecutive points: one voxel for a whole
    wave and longer (all-255 channels, the largest per-wave sums), runs that
    cross wave boundaries, runs of every length 1..70, and a ragged tail."""
    g = w_c1["grid"]
    rng = np.random.default_rng(515)
    centres = rng.uniform(0.05, 0.95, (400, 3)).astype(np.float32)
    lens = np.concatenate([[200, 64, 63, 65, 1], rng.integers(1, 71, 395)])
    pts = np.repeat(centres, lens, axis=0)
    attr = rng.integers(0, 2 ** 32, len(pts), dtype=np.uint64).astype(np.uint32)
    attr[:200] = 0xFFFFFFFF
    for cut in (len(pts), len(pts) - 37):
        p, a = pts[:cut], attr[:cut]
        k, _ = gpu.cga_build(dev(p), g)
        v = gpu.cga_voxel_values(dev(p), dev(a.view(np.int32)), k, g)
        want_k, want_v = oracle.voxel_values(p, a, g)
        assert np.array_equal(u64(k), want_k) and _u32(v).tolist() == want_v.tolist()


@pytest.mark.parametrize("depth", [10, 12])
def test_values_tile_runs(gpu, depth):
    """Voxels whose points span whole 4096-point tiles of the sorted order:
    one voxel of 20,000 points (five tiles and more), runs ending exactly on
    a tile edge and one point past it, many short runs, the points shuffled;
    then a key with no point of the cloud (CGA_EMISMATCH)."""
    g = Grid((0.0, 0.0, 0.0), float(2 ** depth), depth, M)
    rng = np.random.default_rng(517 + depth)
    centres = rng.uniform(0.02, 0.98, (3000, 3)).astype(np.float32)
    lens = np.concatenate([[4096, 4097, 1, 20_000, 4095, 8192], rng.integers(1, 40, 2994)])
    pts = np.repeat(centres, lens, axis=0)
    perm = rng.permutation(len(pts))
    pts = pts[perm]
    attr = rng.integers(0, 2 ** 32, len(pts), dtype=np.uint64).astype(np.uint32)
    k, _ = gpu.cga_build(dev(pts), g)
    v = gpu.cga_voxel_values(dev(pts), dev(attr.view(np.int32)), k, g)
    want_k, want_v = oracle.voxel_values(pts, attr, g)
    assert np.array_equal(u64(k), want_k) and np.array_equal(_u32(v), want_v)
    # the same keys with one extra key no point falls in
    extra = np.array([[0.999, 0.999, 0.0005]], np.float32)
    k2, _ = gpu.cga_build(dev(np.concatenate([pts, extra])), g)
    assert k2.numel() == k.numel() + 1
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_voxel_values(dev(pts), dev(attr.view(np.int32)), k2, g)
    assert e.value.status == gpu.EMISMATCH


@pytest.mark.parametrize("ordered", [False, True])
def test_knn_linear(gpu, w_c1, w_c2s, monkeypatch, ordered):
    """k-NN on LINEAR CGAs (re-keyed to Morton inside the call, positions
    carried along): rows are LINEAR positions, ties broken by the smaller
    LINEAR position, as the oracle does -- c1 (brute force), the c2 sweep,
    a tiny grid full of ties, fewer voxels than k, depth 21."""
    if ordered:
        monkeypatch.setenv("CGA_KNN_ORDER", "1")
    g1 = w_c1["grid"].with_mode(L)
    k1, _ = gpu.cga_build(dev(w_c1["a"]), g1)
    _check_knn(gpu, k1, w_c1["q"], g1, 1, tier="brute")
    g2 = w_c2s["grid"].with_mode(L)
    k2, _ = gpu.cga_build(dev(w_c2s["a"]), g2)
    for k in (1, 8, 16):
        say("knn linear c2s", k, "ordered" if ordered else "")
        _check_knn(gpu, k2, w_c2s["q"], g2, k)
    rng = np.random.default_rng(41)
    g5 = Grid((0.0, 0.0, 0.0), 1.0, 5, L)
    pts = rng.integers(0, 32, (300, 3)).astype(np.float32)
    k5, _ = gpu.cga_build(dev(pts), g5)
    q = np.concatenate([pts[:50], rng.integers(-3, 35, (500, 3)).astype(np.float32)])
    for k in (1, 5, 13, 32):
        _check_knn(gpu, k5, q, g5, k, tier="brute")
    _check_knn(gpu, k5[:3], q[:40], g5, 8, tier="brute")
    g21 = Grid((0.0, 0.0, 0.0), float(2 ** 21), 21, L)
    k21, _ = gpu.cga_build(dev(rng.uniform(0, 1, (20_000, 3)).astype(np.float32)), g21)
    _check_knn(gpu, k21, rng.uniform(0, 1, (700, 3)).astype(np.float32), g21, 4)


# ------------------------------------------------------------------ lookup
def test_binary_lookup(gpu):
    rng = np.random.default_rng(33)
    keys = np.unique(rng.integers(0, 2 ** 48, 500_000, dtype=np.uint64))
    q = np.concatenate([keys[rng.integers(0, len(keys), 100_000)],
                        rng.integers(0, 2 ** 48, 100_000, dtype=np.uint64),
                        np.array([0, 2 ** 64 - 1, keys[0], keys[-1]], np.uint64)])
    r, f = gpu.cga_binary_lookup(dev(keys.view(np.int64)), dev(q.view(np.int64)))
    wr, wf = oracle.lower_bound(keys, q)
    assert np.array_equal(r.cpu().numpy(), wr) and np.array_equal(f.cpu().numpy(), wf)
    r, f = gpu.cga_binary_lookup(dev(keys[:0].view(np.int64)), dev(q[:10].view(np.int64)))
    assert (r.cpu().numpy() == 0).all() and (f.cpu().numpy() == 0).all()


# ------------------------------------------------- device-resident pipeline
@pytest.mark.parametrize("mode", [M, L])
def test_device_count_pipeline_and_repeat(gpu, w_c2s, mode):
    """build -> merge -> project -> kNN with every size left on the device (no
    host sync between calls) equals the synchronous path, twice in a row, on
    both key orders (the LINEAR k-NN re-keys only the device count's keys)."""
    d = w_c2s
    g = d["grid"].with_mode(mode)
    a, b, q = dev(d["a"]), dev(d["b"]), dev(d["q"])
    ref_m, _ = gpu.cga_merge(gpu.cga_build(a, g)[0], gpu.cga_build(b, g)[0], g)
    ref_p, ref_c = gpu.cga_project(ref_m, g, 2)
    ref_i, ref_d = gpu.cga_knn(ref_m, q, g, 8)
    for _ in range(2):
        ws = [gpu.Workspaces() for _ in range(5)]
        cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
        ka, _, _ = gpu.cga_build(a, g, d_n_out=cnt[0:1], sync=False, ws=ws[0])
        kb, _, _ = gpu.cga_build(b, g, d_n_out=cnt[1:2], sync=False, ws=ws[1])
        m, _, _ = gpu.cga_merge(ka, kb, g, d_na=cnt[0:1], d_nb=cnt[1:2], d_n_out=cnt[2:3],
                                sync=False, ws=ws[2])
        p, c, _ = gpu.cga_project(m, g, 2, n=len(a) + len(b), d_n=cnt[2:3], d_n_out=cnt[3:4],
                                  sync=False, ws=ws[3])
        i, dd = gpu.cga_knn(m, q, g, 8, n=len(a) + len(b), d_n=cnt[2:3], ws=ws[4])
        torch.cuda.synchronize()
        n = cnt.cpu().numpy()
        assert n[2] == len(ref_m) and n[3] == len(ref_p)
        assert torch.equal(m[: n[2]], ref_m) and torch.equal(p[: n[3]], ref_p)
        assert torch.equal(c[: n[3]], ref_c)
        assert torch.equal(i, ref_i) and torch.equal(dd, ref_d)


# ----------------------------------------------------- temporal prediction
def _temporal_check(gpu, g, ref, rvals, pred, pvals, window=2, max_iter=20):
    want = oracle.temporal_predict(ref, rvals, pred, pvals, g.depth, g.key_mode, window, max_iter)
    got = gpu.cga_temporal_predict(keys_dev(ref, g), dev(rvals.view(np.int32)), keys_dev(pred, g),
                                   dev(pvals.view(np.int32)), g, window=window, max_iter=max_iter)
    for name in ("ref_assign", "pred_assign", "centroids", "mv", "iters", "match", "residual"):
        np.testing.assert_array_equal(got[name].cpu().numpy(), want[name], err_msg=name)
    np.testing.assert_array_equal(got["sad"].cpu().numpy().view(np.uint32), want["sad"])
    return want


@pytest.fixture(scope="module")
def w_c6s():
    # the moving-object frame pair at 1/10 of the points, on a 512^3 grid
    return gen.c6_frames(n=100_000, depth=9)


@pytest.mark.parametrize("mode", [L, M])
def test_temporal_c6s(gpu, w_c6s, mode):
    d = w_c6s
    g = d["grid"].with_mode(mode)
    ref, rvals = oracle.voxel_values(d["ref"], d["ref_values"], g)
    pred, pvals = oracle.voxel_values(d["pred"], d["pred_values"], g)
    say("temporal c6s", mode, len(ref), len(pred))
    want = _temporal_check(gpu, g, ref, rvals, pred, pvals)
    assert (want["match"] >= 0).mean() > 0.9  # the motion compensation finds most voxels


def test_temporal_edges(gpu):
    rng = np.random.default_rng(91)
    g = Grid((0.0, 0.0, 0.0), 1.0, 5, M)
    ref, _ = oracle.build(rng.integers(0, 32, (400, 3)).astype(np.float32), g)
    pred, _ = oracle.build(rng.integers(0, 32, (300, 3)).astype(np.float32), g)
    rvals = rng.integers(0, 2 ** 32, len(ref), dtype=np.uint64).astype(np.uint32)
    pvals = rng.integers(0, 2 ** 32, len(pred), dtype=np.uint64).astype(np.uint32)
    for window, max_iter in ((0, 1), (1, 3), (2, 50), (5, 1000)):
        _temporal_check(gpu, g, ref, rvals, pred, pvals, window, max_iter)
    gl = g.with_mode(L)
    lref, lr = oracle.voxel_values(oracle.decode(ref, 5, M).astype(np.float32), rvals, gl)
    lpred, lp = oracle.voxel_values(oracle.decode(pred, 5, M).astype(np.float32), pvals, gl)
    _temporal_check(gpu, gl, lref, lr, lpred, lp, 3, 20)
    _temporal_check(gpu, gl, lref[:1], lr[:1], lpred, lp, 2, 20)  # one reference voxel
    _temporal_check(gpu, gl, lref, lr, lpred[:1], lp[:1], 2, 20)  # one predicted voxel
    e = np.zeros(0, np.uint64)
    _temporal_check(gpu, gl, e, lr[:0], lpred, lp, 2, 20)  # empty reference: no matches
    _temporal_check(gpu, gl, lref, lr, e, lp[:0], 2, 20)  # empty predicted frame
    with pytest.raises(gpu.CgaError) as err:
        gpu.cga_temporal_predict(keys_dev(lref, gl), dev(lr.view(np.int32)), keys_dev(lpred, gl),
                                 dev(lp.view(np.int32)), gl, window=16)
    assert err.value.status == gpu.EINVAL
