"""Pins of the CPU oracle against facts fixed by the paper and by mathematics:
closed forms, hand-worked Table II examples, independent library routes,
invariants of the set operations, and brute force on tiny inputs.

A plausible mistake anywhere in the oracle (a swapped Morton bit, a fused or
double-precision quantizer, a dropped duplicate, a wrong tie-break, a missed
far side in the kd-tree, a gradient sign) fails at least one test here.
"""
import json
import os

import numpy as np
import pytest

import gen
import oracle
from gen import Grid

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M, L = oracle.MORTON, oracle.LINEAR


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def int_grid(depth, mode):
    """Identity grid for integer-valued float coordinates: voxel = coordinate."""
    return Grid((0.0, 0.0, 0.0), 1.0, depth, mode)


# ------------------------------------------------------------- quantization
class TestQuantize:
    g = Grid((0.0, 0.0, 0.0), 1024.0, 10, M)

    def test_exact_dyadic(self):
        i = np.arange(1024, dtype=np.float64)
        p = np.stack([i / 1024, i[::-1] / 1024, (i * 7 % 1024) / 1024], 1).astype(np.float32)
        v = oracle.quantize(p, self.g)
        assert (v[:, 0] == i).all() and (v[:, 1] == i[::-1]).all()
        assert (v[:, 2] == i * 7 % 1024).all()

    def test_just_below_one_and_clamps(self):
        p = np.array([[1 - 2 ** -24, 0.0, 0.5], [-1e-7, 1.0, 5.0], [-3.0, 1e30, -1e30]], np.float32)
        v = oracle.quantize(p, self.g)
        assert v.tolist() == [[1023, 0, 512], [0, 1023, 1023], [0, 1023, 0]]

    def test_subtract_is_rounded_before_multiply(self):
        # fl32(1 - 2^-25) ties to even = 1.0, so the voxel is 512; the exact
        # value (1 - 2^-25) * 512 would floor to 511.
        g = Grid((2.0 ** -25, 0.0, 0.0), 512.0, 10, M)
        v = oracle.quantize(np.array([[1.0, 0.0, 0.0]], np.float32), g)
        assert v[0, 0] == 512

    def test_matches_ieee_float32_arithmetic(self):
        rng = np.random.default_rng(5)
        p = rng.uniform(-10, 110, (20000, 3)).astype(np.float32)
        o = np.float32([-3.3, 0.7, 1.1])
        s = np.float32(17.123)
        g = Grid(tuple(float(x) for x in o), float(s), 11, M)
        t = (p - o).astype(np.float32)
        u = (t * s).astype(np.float32)
        want = np.clip(np.floor(u), 0, 2 ** 11 - 1).astype(np.uint32)
        assert (oracle.quantize(p, g) == want).all()

    @pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
    def test_nonfinite_is_error(self, bad):
        p = np.array([[0.5, 0.5, 0.5], [0.1, bad, 0.2]], np.float32)
        with pytest.raises(oracle.NonFinite):
            oracle.quantize(p, self.g)
        with pytest.raises(oracle.NonFinite):
            oracle.build(p, self.g)


# ------------------------------------------------------------------- keys
def _spread3(v):
    """Test-local magic-number bit spread (a different algorithm from the
    oracle's per-bit loop): bit b -> bit 3b, for values below 2^21."""
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


class TestKeys:
    def test_morton_hand_values(self):
        vox = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [2, 0, 0], [3, 3, 3], [0, 2, 1]]
        assert oracle.encode(vox, 10, M).tolist() == [4, 2, 1, 7, 32, 63, 16 + 1]

    @pytest.mark.parametrize("d", [1, 5, 10, 11, 16, 21])
    def test_all_ones(self, d):
        m = 2 ** d - 1
        assert int(oracle.encode([[m, m, m]], d, M)[0]) == 2 ** (3 * d) - 1
        assert int(oracle.encode([[m, m, m]], d, L)[0]) == 2 ** (3 * d) - 1

    @pytest.mark.parametrize("d", [3, 10, 12, 16, 21])
    def test_matches_magic_spread_and_roundtrips(self, d):
        rng = np.random.default_rng(d)
        v = rng.integers(0, 2 ** d, (5000, 3)).astype(np.uint32)
        want = (_spread3(v[:, 0]) << np.uint64(2)) | (_spread3(v[:, 1]) << np.uint64(1)) | _spread3(v[:, 2])
        k = oracle.encode(v, d, M)
        assert (k == want).all()
        assert (oracle.decode(k, d, M) == v).all()
        kl = oracle.encode(v, d, L)
        assert (oracle.decode(kl, d, L) == v).all()

    def test_morton_prefix_is_octree_cell(self):
        d = 12
        rng = np.random.default_rng(1)
        v = rng.integers(0, 2 ** d, (3000, 3)).astype(np.uint32)
        k = oracle.encode(v, d, M)
        for lvl in range(d + 1):
            parent = oracle.encode(v >> lvl, d, M)
            assert (k >> np.uint64(3 * lvl) == parent).all()

    def test_linear_order_is_lexicographic(self):
        d = 7
        rng = np.random.default_rng(2)
        v = rng.integers(0, 2 ** d, (4000, 3)).astype(np.uint32)
        order_lex = np.lexsort((v[:, 2], v[:, 1], v[:, 0]))
        k = oracle.encode(v, d, L)
        assert (np.sort(k) == k[order_lex]).all()

    def test_key2(self):
        assert oracle.encode2([1, 0, 3], [0, 1, 3], 4, M).tolist() == [2, 1, 15]
        assert oracle.encode2([1, 0, 3], [0, 1, 3], 4, L).tolist() == [16, 1, 51]


# ------------------------------------------------------------------ build
def _per_point_keys(xyz, grid):
    return oracle.encode(oracle.quantize(xyz, grid), grid.depth, grid.key_mode)


class TestBuild:
    @pytest.mark.parametrize("mode", [M, L])
    def test_equals_sort_unique(self, mode):
        d = gen.c1_spheres(n=20000, nq=1)
        g = d["grid"].with_mode(mode)
        keys, counts = oracle.build(d["a"], g)
        uk, uc = np.unique(_per_point_keys(d["a"], g), return_counts=True)
        assert (keys == uk).all() and (counts == uc).all()
        assert counts.sum() == len(d["a"])

    def test_heavy_duplicates(self):
        rng = np.random.default_rng(3)
        xyz = rng.integers(0, 4, (5000, 3)).astype(np.float32)
        keys, counts = oracle.build(xyz, int_grid(3, M))
        assert len(keys) <= 64 and counts.sum() == 5000
        uk, uc = np.unique(_per_point_keys(xyz, int_grid(3, M)), return_counts=True)
        assert (keys == uk).all() and (counts == uc).all()

    def test_empty(self):
        keys, counts = oracle.build(np.zeros((0, 3), np.float32), int_grid(4, M))
        assert len(keys) == 0 and len(counts) == 0

    @pytest.mark.parametrize("name", ["soldier", "gt_madame"])
    def test_table2_arrays(self, name):
        pts = np.array(_gold("table2_points.json")[name], np.float32)
        want = _gold("table2_derived.json")[name + "_arrays"]
        for mode in (M, L):
            keys, counts = oracle.build(pts, int_grid(8, mode))
            assert len(keys) == 6 and (counts == 1).all()
            arr = oracle.arrays(keys, 8, mode)
            for k, v in want.items():
                assert arr[k].tolist() == v, (name, mode, k)

    def test_arrays_structure_random(self):
        rng = np.random.default_rng(4)
        d = 6
        xyz = rng.integers(0, 2 ** d, (3000, 3)).astype(np.float32)
        keys, _ = oracle.build(xyz, int_grid(d, L))
        arr = oracle.arrays(keys, d, L)
        vox = oracle.decode(keys, d, L)
        # CSR expansion of the three levels reproduces the voxel set in order
        xp, yp = arr["x_pointer"], arr["y_pointer"]
        x_rep = np.repeat(arr["x_index"], np.diff(xp))
        assert len(x_rep) == len(arr["y_index"])
        xs = np.repeat(x_rep, np.diff(yp))
        ys = np.repeat(arr["y_index"], np.diff(yp))
        assert (np.stack([xs, ys, arr["z_index"]], 1) == vox).all()
        assert xp[-1] == len(arr["y_index"]) and yp[-1] == len(keys)
        assert len(np.unique(arr["x_index"])) == len(arr["x_index"])


# ------------------------------------------------------------------ merge
class TestMerge:
    def _two(self, seed, n=3000, d=6):
        rng = np.random.default_rng(seed)
        a = rng.integers(0, 2 ** d, (n, 3)).astype(np.float32)
        b = rng.integers(0, 2 ** d, (n, 3)).astype(np.float32)
        return a, b

    @pytest.mark.parametrize("mode", [M, L])
    def test_union_invariants(self, mode):
        a, b = self._two(7)
        g = int_grid(6, mode)
        ka, _ = oracle.build(a, g)
        kb, _ = oracle.build(b, g)
        u, src = oracle.merge(ka, kb, 6, mode)
        assert (u == np.union1d(ka, kb)).all()
        u2, src2 = oracle.merge(kb, ka, 6, mode)
        assert (u2 == u).all()
        assert ((src2 == 3) == (src == 3)).all() and ((src2 == 1) == (src == 2)).all()
        inter = int((src == 3).sum())
        assert len(u) == len(ka) + len(kb) - inter
        assert inter == len(np.intersect1d(ka, kb))
        assert np.isin(ka, u).all() and np.isin(kb, u).all()
        uu, s = oracle.merge(ka, ka, 6, mode)
        assert (uu == ka).all() and (s == 3).all()
        ue, s = oracle.merge(ka, np.zeros(0, np.uint64), 6, mode)
        assert (ue == ka).all() and (s == 1).all()

    def test_table2_merge(self):
        pts = _gold("table2_points.json")
        g = int_grid(8, M)
        ka, _ = oracle.build(np.array(pts["soldier"], np.float32), g)
        kb, _ = oracle.build(np.array(pts["gt_madame"], np.float32), g)
        u, src = oracle.merge(ka, kb, 8, M)
        assert len(u) == _gold("table2_derived.json")["merge_size"]
        assert (src[np.isin(u, ka)] == 1).all() and (src[np.isin(u, kb)] == 2).all()


# ------------------------------------------------------------- projection
class TestProject:
    @pytest.mark.parametrize("mode", [M, L])
    @pytest.mark.parametrize("axis", [0, 1, 2])
    def test_invariants(self, mode, axis):
        rng = np.random.default_rng(11 + axis)
        d = 5
        a = rng.integers(0, 2 ** d, (2000, 3)).astype(np.float32)
        b = rng.integers(0, 2 ** d, (2000, 3)).astype(np.float32)
        g = int_grid(d, mode)
        ka, _ = oracle.build(a, g)
        kb, _ = oracle.build(b, g)
        pa, ca = oracle.project(ka, d, mode, axis)
        pb, _ = oracle.project(kb, d, mode, axis)
        u, _ = oracle.merge(ka, kb, d, mode)
        pu, _ = oracle.project(u, d, mode, axis)
        assert (pu == np.union1d(pa, pb)).all()  # P(A u B) = P(A) u P(B)
        assert ca.sum() == len(ka) and len(pa) <= len(ka)
        # independent route: drop the coordinate, encode, unique with counts
        vox = oracle.decode(ka, d, mode)
        keep = [i for i in range(3) if i != axis]
        k2 = oracle.encode2(vox[:, keep[0]], vox[:, keep[1]], d, mode)
        uk, uc = np.unique(k2, return_counts=True)
        assert (pa == uk).all() and (ca == uc).all()

    def test_linear_drop_z_is_xy_arrays(self):
        rng = np.random.default_rng(12)
        d = 6
        a = rng.integers(0, 2 ** d, (4000, 3)).astype(np.float32)
        keys, _ = oracle.build(a, int_grid(d, L))
        arr = oracle.arrays(keys, d, L)
        p, c = oracle.project(keys, d, L, 2)
        xs = np.repeat(arr["x_index"], np.diff(arr["x_pointer"]))
        assert (p == oracle.encode2(xs, arr["y_index"], d, L)).all()
        assert (c == np.diff(arr["y_pointer"])).all()

    def test_table2_projection(self):
        pts = np.array(_gold("table2_points.json")["soldier"], np.float32)
        want = _gold("table2_derived.json")
        for mode in (M, L):
            keys, _ = oracle.build(pts, int_grid(8, mode))
            for axis, name in ((2, "soldier_project_drop_z"), (1, "soldier_project_drop_y")):
                p, c = oracle.project(keys, 8, mode, axis)
                pix = np.array(want[name]["pixels"], np.uint32)
                wk = oracle.encode2(pix[:, 0], pix[:, 1], 8, mode)
                order = np.argsort(wk)
                assert (p == wk[order]).all()
                assert (c == np.array(want[name]["counts"])[order]).all()
            p, c = oracle.project(keys, 8, mode, 0)
            assert len(p) == want["soldier_project_drop_x_size"] and (c == 1).all()


# --------------------------------------------------------------------- kNN
class TestKnn:
    def test_table2_tie(self):
        pts = np.array(_gold("table2_points.json")["soldier"], np.float32)
        w = _gold("table2_derived.json")["soldier_knn"]
        for mode in (M, L):
            g = int_grid(8, mode)
            keys, _ = oracle.build(pts, g)
            q = np.array([w["query"]], np.float32)
            for fn in (oracle.knn_brute, oracle.knn_kdtree):
                idx, d2 = fn(keys, q, g, w["k"])
                got = oracle.decode(keys[idx[0]], 8, mode).tolist()
                assert got == w["neighbours"] and d2[0].tolist() == w["d2"]

    @pytest.mark.parametrize("mode", [M, L])
    @pytest.mark.parametrize("k", [1, 3, 8, 16])
    def test_brute_matches_direct_and_kdtree(self, mode, k):
        rng = np.random.default_rng(20 + k)
        d = 5  # small grid: many exact distance ties
        pts = rng.integers(0, 2 ** d, (600, 3)).astype(np.float32)
        g = int_grid(d, mode)
        keys, _ = oracle.build(pts, g)
        q = rng.integers(0, 2 ** d, (300, 3)).astype(np.float32)
        idx, d2 = oracle.knn_brute(keys, q, g, k)
        # direct restatement with numpy: lexsort by (d2, index)
        vox = oracle.decode(keys, d, mode).astype(np.int64)
        qv = q.astype(np.int64)
        for j in range(len(q)):
            dd = ((vox - qv[j]) ** 2).sum(1)
            order = np.lexsort((np.arange(len(vox)), dd))[:k]
            assert (idx[j] == order).all() and (d2[j] == dd[order]).all()
        ik, dk = oracle.knn_kdtree(keys, q, g, k)
        assert (ik == idx).all() and (dk == d2).all()

    def test_distances_match_scipy(self):
        from scipy.spatial import cKDTree
        rng = np.random.default_rng(30)
        pts = rng.integers(0, 1000, (5000, 3)).astype(np.float32)
        g = int_grid(10, M)
        keys, _ = oracle.build(pts, g)
        q = rng.integers(0, 1000, (500, 3)).astype(np.float32)
        _, d2 = oracle.knn_kdtree(keys, q, g, 8)
        vox = oracle.decode(keys, 10, M).astype(np.float64)
        dist, _ = cKDTree(vox).query(q.astype(np.float64), k=8)
        assert np.array_equal(np.rint(dist ** 2).astype(np.uint64), d2)

    def test_occupied_and_padding(self):
        rng = np.random.default_rng(31)
        pts = rng.integers(0, 64, (50, 3)).astype(np.float32)
        g = int_grid(6, M)
        keys, _ = oracle.build(pts, g)
        idx, d2 = oracle.knn_brute(keys, pts, g, 1)
        assert (d2[:, 0] == 0).all()
        assert (keys[idx[:, 0]] == oracle.encode(pts.astype(np.uint32), 6, M)).all()
        u = len(keys)
        idx, d2 = oracle.knn_kdtree(keys, pts[:5], g, u + 3)
        assert (np.sort(idx[:, :u], 1) == np.arange(u)).all()
        assert (idx[:, u:] == -1).all() and (d2[:, u:] == np.iinfo(np.uint64).max).all()
        idx, d2 = oracle.knn_brute(np.zeros(0, np.uint64), pts[:2], g, 2)
        assert (idx == -1).all()

    @pytest.mark.parametrize("mode", [M, L])
    def test_paper_cga_nn_matches_brute(self, mode):
        rng = np.random.default_rng(40 + mode)
        d = 6
        pts = rng.integers(0, 2 ** d, (800, 3)).astype(np.float32)
        g = int_grid(d, mode)
        keys, _ = oracle.build(pts, g)
        arr = oracle.arrays(keys, d, mode)
        qv = rng.integers(0, 2 ** d, (400, 3)).astype(np.uint32)
        pos, dd = oracle.nn_cga(arr, qv, d, mode)
        idx, d2 = oracle.knn_brute(keys, qv.astype(np.float32), g, 1)
        assert (dd == d2[:, 0]).all()
        # positions are in (x, y, z) order; map the brute-force answer there
        lin = oracle.encode(oracle.decode(keys[idx[:, 0]], d, mode), d, L)
        lin_sorted = np.sort(oracle.encode(oracle.decode(keys, d, mode), d, L))
        assert (np.searchsorted(lin_sorted, lin) == pos).all()

    def test_paper_nn_hand_example(self):
        """Voxels (0,0,0), (2,0,0), (2,5,1): the nearest-x walk from (3,0,4)
        lands on (2,0,0) (epsilon^2 = 17), and the box search then finds
        nothing closer; from (2,4,1) the walk meets (2,5,1) at distance 1."""
        g = int_grid(3, L)
        keys, _ = oracle.build(np.array([[0, 0, 0], [2, 0, 0], [2, 5, 1]], np.float32), g)
        arr = oracle.arrays(keys, 3, L)
        pos, dd = oracle.nn_cga(arr, np.array([[3, 0, 4], [2, 4, 1], [0, 0, 0]], np.uint32), 3, L)
        assert pos.tolist() == [1, 2, 0] and dd.tolist() == [17, 1, 0]

    def test_nonfinite_query(self):
        keys, _ = oracle.build(np.zeros((1, 3), np.float32), int_grid(4, M))
        with pytest.raises(oracle.NonFinite):
            oracle.knn_brute(keys, np.array([[np.nan, 0, 0]], np.float32), int_grid(4, M), 1)


class TestPaperLookup:
    """Three-level lookup on the five arrays (Section V-A) against membership
    and rank in the sorted key array (a definition that uses no array but the
    keys)."""

    @pytest.mark.parametrize("d", [3, 7])
    def test_matches_key_rank(self, d):
        rng = np.random.default_rng(60 + d)
        pts = rng.integers(0, 2 ** d, (3000, 3)).astype(np.float32)
        g = int_grid(d, L)
        keys, _ = oracle.build(pts, g)
        arr = oracle.arrays(keys, d, L)
        qv = np.concatenate([oracle.decode(keys[rng.integers(0, len(keys), 500)], d, L),
                             rng.integers(0, 2 ** d, (500, 3))]).astype(np.uint32)
        pos = oracle.lookup_cga(arr, qv)
        rank, found = oracle.lower_bound(keys, oracle.encode(qv, d, L))
        assert (pos == np.where(found.astype(bool), rank, -1)).all()
        assert (pos[:500] >= 0).all()

    def test_hand_example(self):
        # voxels (1,2,3), (1,2,5), (1,4,0), (6,0,0): X_index [1, 6], X_pointer
        # [0, 2, 3], Y_index [2, 4, 0], Y_pointer [0, 2, 3, 4], Z_index [3, 5, 0, 0]
        g = int_grid(3, L)
        keys, _ = oracle.build(np.array([[1, 2, 3], [1, 2, 5], [1, 4, 0], [6, 0, 0]],
                                        np.float32), g)
        arr = oracle.arrays(keys, 3, L)
        assert arr["x_index"].tolist() == [1, 6] and arr["x_pointer"].tolist() == [0, 2, 3]
        assert arr["y_pointer"].tolist() == [0, 2, 3, 4]
        q = np.array([[1, 2, 5], [1, 4, 0], [6, 0, 0], [1, 2, 4], [1, 3, 0], [2, 0, 0],
                      [6, 0, 1], [0, 0, 0]], np.uint32)
        assert oracle.lookup_cga(arr, q).tolist() == [1, 2, 3, -1, -1, -1, -1, -1]
        empty = oracle.arrays(np.zeros(0, np.uint64), 3, L)
        assert oracle.lookup_cga(empty, q[:2]).tolist() == [-1, -1]


# ----------------------------------------------------------------- lookup
def test_lower_bound_matches_searchsorted():
    rng = np.random.default_rng(50)
    keys = np.unique(rng.integers(0, 2 ** 48, 100000).astype(np.uint64))
    q = np.concatenate([keys[rng.integers(0, len(keys), 5000)],
                        rng.integers(0, 2 ** 48, 5000).astype(np.uint64),
                        np.array([0, 2 ** 64 - 1], np.uint64)])
    rank, found = oracle.lower_bound(keys, q)
    assert (rank == np.searchsorted(keys, q, side="left")).all()
    assert (found.astype(bool) == np.isin(q, keys)).all()
    assert found[:5000].all()


# -------------------------------------------------------------- MLP grads
def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(60)
    p = rng.normal(0, 1, 49)
    x = rng.uniform(0, 1, 300)
    t = np.sort(rng.uniform(0, 1, 300))
    loss, g, kinks = oracle.mlp_loss_grad(p, x, t)
    assert kinks == 0
    # direct loss restatement
    f = (np.maximum(0, np.outer(x, p[:16]) + p[16:32]) * p[32:48]).sum(1) + p[48]
    assert abs(loss - ((f - t) ** 2).mean()) < 1e-12
    h = 1e-6
    for j in range(49):
        e = np.zeros(49)
        e[j] = h
        num = (oracle.mlp_loss_grad(p + e, x, t)[0] - oracle.mlp_loss_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(num - g[j]) <= 1e-6 * max(1.0, abs(g[j])), j


# ------------------------------------------------------------ occupancy codes
def _decode_occupancy(codes, depth):
    """Rebuild the key set from occupancy codes, root first, level by level:
    the decoder the paper describes (only the codes are needed)."""
    prefixes, t = [0], 0
    for _ in range(depth):
        nxt = []
        for p in prefixes:
            c = int(codes[t])
            t += 1
            nxt.extend(p * 8 + o for o in range(8) if (c >> o) & 1)
        prefixes = nxt
    assert t == len(codes)
    return np.array(prefixes, dtype=np.uint64)


def test_occupancy_hand_examples():
    # depth 1: voxels in octants 0 and 7 of the root
    codes, counts = oracle.occupancy(np.array([0, 7], np.uint64), 1)
    assert codes.tolist() == [0x81] and counts.tolist() == [2, 1]
    # depth 2: voxel 0 (cell 0, octant 0) and voxel 63 (cell 7, octant 7)
    codes, counts = oracle.occupancy(np.array([0, 63], np.uint64), 2)
    assert codes.tolist() == [0x81, 0x01, 0x80] and counts.tolist() == [2, 2, 1]
    # one voxel at the far corner of a depth-3 grid: one path of octant 7
    codes, counts = oracle.occupancy(np.array([511], np.uint64), 3)
    assert codes.tolist() == [0x80, 0x80, 0x80] and counts.tolist() == [1, 1, 1, 1]


@pytest.mark.parametrize("depth,n", [(1, 5), (2, 30), (4, 300), (7, 5000), (10, 20000)])
def test_occupancy_decodes_to_the_keys(depth, n):
    rng = np.random.default_rng(depth * 1000 + n)
    keys = np.unique(rng.integers(0, 8 ** depth, n, dtype=np.uint64))
    codes, counts = oracle.occupancy(keys, depth)
    np.testing.assert_array_equal(_decode_occupancy(codes, depth), keys)
    # one code per occupied cell of levels depth .. 1, whose set bits are the
    # occupied cells one level down
    assert len(codes) == counts[1:].sum() and counts[0] == len(keys) and counts[depth] == 1
    pc = np.unpackbits(codes[:, None], axis=1).sum(1)
    off = 0
    for L in range(depth, 0, -1):
        assert pc[off:off + counts[L]].sum() == counts[L - 1]
        off += counts[L]


def test_occupancy_of_the_c1_cloud_decodes():
    d = gen.c1_spheres(n=20000)
    keys, _ = oracle.build(d["a"], d["grid"])
    codes, _ = oracle.occupancy(keys, d["grid"].depth)
    np.testing.assert_array_equal(_decode_occupancy(codes, d["grid"].depth), keys)


# ------------------------------------------------------------ attribute values
def _pack(rgb):
    rgb = np.asarray(rgb, np.uint32)
    return rgb[:, 0] | (rgb[:, 1] << 8) | (rgb[:, 2] << 16)


def _soldier():
    here = os.path.join(os.path.dirname(__file__), "golden")
    pts = np.array(json.load(open(os.path.join(here, "table2_points.json")))["soldier"], np.float32)
    rgb = json.load(open(os.path.join(here, "table2_colors.json")))["soldier_rgb"]
    return pts, _pack(rgb)


def test_values_table2_soldier():
    pts, col = _soldier()
    # one voxel per printed point: each keeps its own colour
    g = Grid((0.0, 0.0, 0.0), 1.0, 8, gen.KEY_MORTON)
    keys, vals = oracle.voxel_values(pts, col, g)
    want = {int(k): int(c) for k, c in zip(oracle.encode(oracle.quantize(pts, g), 8, 0), col)}
    assert {int(k): int(v) for k, v in zip(keys, vals)} == want
    # at scale 1/4 the first four rows share voxel (31, 3, 39) -- all
    # (82, 73, 67) -- and the last two share (31, 4, 38): (79, 72, 67) and
    # (83, 77, 73) average to (81, 74.5 -> 75, 70)
    g4 = Grid((0.0, 0.0, 0.0), 0.25, 8, gen.KEY_MORTON)
    keys, vals = oracle.voxel_values(pts, col, g4)
    got = {tuple(int(c) for c in oracle.decode(np.array([k], np.uint64), 8, 0)[0]): int(v)
           for k, v in zip(keys, vals)}
    assert got == {(31, 3, 39): int(_pack([[82, 73, 67]])[0]),
                   (31, 4, 38): int(_pack([[81, 75, 70]])[0])}


def test_values_rounding_and_invariances():
    g = Grid((0.0, 0.0, 0.0), 1.0, 4, gen.KEY_MORTON)
    one = np.zeros((2, 3), np.float32)  # two points, one voxel
    _, v = oracle.voxel_values(one, np.array([0x000000FF, 0x00000001], np.uint32), g)
    assert v.tolist() == [128]          # (255 + 1) / 2
    _, v = oracle.voxel_values(one, np.array([0x01020301, 0x01030402], np.uint32), g)
    assert v.tolist() == [0x01030402]   # halves round up: 1.5 -> 2, 3.5 -> 4, 2.5 -> 3
    rng = np.random.default_rng(7)
    xyz = rng.uniform(0, 16, (5000, 3)).astype(np.float32)
    attr = gen.attributes(7, 1, len(xyz))
    k1, v1 = oracle.voxel_values(xyz, attr, g)
    perm = rng.permutation(len(xyz))
    k2, v2 = oracle.voxel_values(xyz[perm], attr[perm], g)
    assert np.array_equal(k1, k2) and np.array_equal(v1, v2)   # order of points is irrelevant
    kb, _ = oracle.build(xyz, g)
    assert np.array_equal(k1, kb)                              # same voxels as the build
    kc, vc = oracle.voxel_values(xyz, np.full(len(xyz), 0x11223344, np.uint32), g)
    assert (vc == 0x11223344).all()                            # constant colour stays


def test_merge_values_policies():
    rng = np.random.default_rng(8)
    ka = np.unique(rng.integers(0, 4096, 900).astype(np.uint64))
    kb = np.unique(rng.integers(0, 4096, 900).astype(np.uint64))
    va = gen.attributes(8, 1, len(ka))
    vb = gen.attributes(8, 2, len(kb))
    m, _ = oracle.merge(ka, kb, 4, 0)
    for pol in (oracle.BASE, oracle.AVERAGE):
        k, v = oracle.merge_values(ka, va, kb, vb, pol)
        assert np.array_equal(k, m)
    kbase, vbase = oracle.merge_values(ka, va, kb, vb, oracle.BASE)
    kavg, vavg = oracle.merge_values(ka, va, kb, vb, oracle.AVERAGE)
    both = np.intersect1d(ka, kb)
    ia, ib, ix = (np.searchsorted(ka, both), np.searchsorted(kb, both), np.searchsorted(kbase, both))
    assert np.array_equal(vbase[ix], va[ia])                   # base wins
    ch = lambda x, c: (x >> (8 * c)) & 0xFF
    for c in range(4):
        assert np.array_equal(ch(vavg[ix], c), (ch(va[ia], c) + ch(vb[ib], c) + 1) // 2)
    only_b = np.setdiff1d(kb, ka)
    assert np.array_equal(vbase[np.searchsorted(kbase, only_b)], vb[np.searchsorted(kb, only_b)])
    # the average is symmetric; merging with an empty cloud changes nothing
    k2, v2 = oracle.merge_values(kb, vb, ka, va, oracle.AVERAGE)
    assert np.array_equal(k2, kavg) and np.array_equal(v2, vavg)
    k3, v3 = oracle.merge_values(ka, va, ka[:0], va[:0], oracle.AVERAGE)
    assert np.array_equal(k3, ka) and np.array_equal(v3, va)


# ------------------------------------------------------- temporal prediction
def _chan(v):
    v = np.asarray(v, np.uint32)
    return np.stack([(v >> np.uint32(8 * c)) & np.uint32(0xFF) for c in range(4)], -1).astype(np.int64)


class TestTemporal:
    """Temporal prediction steps (Section V-D) against what fixes them: the
    k-means fixed point (nearest-centre assignment, centres = means), the
    bounding-box corner seeds, exact recovery of a known translation, and the
    SAD-minimality of every match over its window."""

    def _frame(self, rng, d, n):
        g = int_grid(d, M)
        keys, _ = oracle.build(rng.integers(0, 2 ** d, (n, 3)).astype(np.float32), g)
        return keys

    def test_kmeans_fixed_point_and_seeds(self):
        rng = np.random.default_rng(80)
        d = 7
        keys = self._frame(rng, d, 3000)
        vals = rng.integers(0, 2 ** 32, len(keys), dtype=np.uint64).astype(np.uint32)
        vox = oracle.decode(keys, d, M).astype(np.float64)
        out = oracle.temporal_predict(keys, vals, keys, vals, d, M, 1, 200)
        c = out["centroids"][0]
        dd = ((vox[:, None, :] - c[None]) ** 2)
        dist = (dd[..., 0] + dd[..., 1]) + dd[..., 2]
        assert (out["ref_assign"] == np.argmin(dist, 1)).all()  # nearest centre, ties low
        assert out["iters"][0] < 200  # converged: every centre is the mean of its voxels
        vi = oracle.decode(keys, d, M).astype(np.int64)
        for k in range(8):
            sel = out["ref_assign"] == k
            if sel.any():
                assert (c[k] == vi[sel].sum(0) / sel.sum()).all()
        one = oracle.temporal_predict(keys, vals, keys, vals, d, M, 1, 1)
        lo, hi = vi.min(0), vi.max(0)
        for k in range(8):
            corner = [hi[a] if (k >> (2 - a)) & 1 else lo[a] for a in range(3)]
            assert one["centroids"][0][k].tolist() == corner
        assert one["iters"].tolist() == [1, 1]

    def test_translation_recovered(self):
        rng = np.random.default_rng(81)
        d = 8
        vox = rng.integers(20, 200, (4000, 3))
        t = np.array([3, -5, 2])
        ga = int_grid(d, L)
        ref, _ = oracle.build(vox.astype(np.float32), ga)
        pred, _ = oracle.build((vox + t).astype(np.float32), ga)
        rv = oracle.decode(ref, d, L).astype(np.int64)
        ref_vals = (rv[:, 0] * 7 + rv[:, 1] * 3 + rv[:, 2]).astype(np.uint32) * np.uint32(0x010203)
        pv = oracle.decode(pred, d, L).astype(np.int64) - t
        pred_vals = (pv[:, 0] * 7 + pv[:, 1] * 3 + pv[:, 2]).astype(np.uint32) * np.uint32(0x010203)
        out = oracle.temporal_predict(ref, ref_vals, pred, pred_vals, d, L, 2, 50)
        assert (out["mv"] == t).all()
        assert (out["ref_assign"] == out["pred_assign"]).all()  # pred is in key order too
        assert (out["sad"] == 0).all() and (out["residual"] == 0).all()
        assert (out["match"] == np.arange(len(ref))).all()

    def test_match_is_window_sad_minimum(self):
        rng = np.random.default_rng(82)
        d, w = 5, 2
        ref = self._frame(rng, d, 600)
        pred = self._frame(rng, d, 300)
        rvals = rng.integers(0, 2 ** 32, len(ref), dtype=np.uint64).astype(np.uint32)
        pvals = rng.integers(0, 2 ** 32, len(pred), dtype=np.uint64).astype(np.uint32)
        out = oracle.temporal_predict(ref, rvals, pred, pvals, d, M, w, 30)
        rvox = oracle.decode(ref, d, M).astype(np.int64)
        pvox = oracle.decode(pred, d, M).astype(np.int64)
        rch, pch = _chan(rvals), _chan(pvals)
        recon = pvox - out["mv"][out["pred_assign"]]
        for i in range(len(pred)):
            inwin = (np.abs(rvox - recon[i]) <= w).all(1)
            sads = np.abs(rch - pch[i]).sum(1)
            if not inwin.any() or (recon[i] < 0).any() or (recon[i] >= 2 ** d).any():
                assert out["match"][i] == -1 and out["sad"][i] == 2 ** 32 - 1
                assert (out["residual"][i] == pch[i]).all()
                continue
            j = out["match"][i]
            assert inwin[j] and out["sad"][i] == sads[j] == sads[inwin].min()
            l1 = np.abs(rvox - recon[i]).sum(1)
            tied = inwin & (sads == sads[j])
            assert l1[j] == l1[tied].min() and j == np.flatnonzero(tied & (l1 == l1[j]))[0]
            assert (out["residual"][i] == pch[i] - rch[j]).all()

    def test_hand_example(self):
        """Reference voxels (4,4,4), (5,4,4), (7,4,4) with red 250, red 190,
        green 250.  All four x-min corners are (4,4,4): the first pass puts
        (4,4,4) and (5,4,4) in cluster 0 (ties to the lower cluster), (7,4,4)
        in cluster 4; cluster 0 moves to x = 4.5, so the second pass gives
        (4,4,4) to the empty cluster 1 still sitting on the corner, and the
        third repeats: centroids (5,4,4), (4,4,4), ..., (7,4,4).  A one-voxel
        predicted frame at (4,4,4) stays in cluster 0 with centroid 4, so its
        motion vector is -1 on x and it is matched from (5,4,4): with window
        1, red 190 there (SAD 10) beats the co-located red 250 (SAD 50)."""
        g = int_grid(4, L)
        ref, _ = oracle.build(np.array([[4, 4, 4], [5, 4, 4], [7, 4, 4]], np.float32), g)
        rvals = np.array([250, 190, 250 << 8], np.uint32)  # channel 0 in the low byte
        pred, _ = oracle.build(np.array([[4, 4, 4]], np.float32), g)
        out = oracle.temporal_predict(ref, rvals, pred, np.array([200], np.uint32), 4, L, 1, 5)
        assert out["ref_assign"].tolist() == [1, 0, 4] and out["iters"].tolist() == [3, 2]
        assert out["centroids"][0][:2].tolist() == [[5, 4, 4], [4, 4, 4]]
        assert out["centroids"][0][4].tolist() == [7, 4, 4]
        assert out["mv"].tolist() == [[-1, 0, 0]] + [[0, 0, 0]] * 3 + [[-3, 0, 0]] * 4
        assert out["match"].tolist() == [1] and out["sad"].tolist() == [10]
        assert out["residual"].tolist() == [[10, 0, 0, 0]]
        # (0,0,0) of value 7: motion vector (0,0,0) - (5,4,4) moves it to
        # (5,4,4); SAD 183 from (5,4,4) beats 243 from (4,4,4)
        far, _ = oracle.build(np.array([[0, 0, 0]], np.float32), g)
        out = oracle.temporal_predict(ref, rvals, far, np.array([7], np.uint32), 4, L, 1, 5)
        assert out["mv"][0].tolist() == [-5, -4, -4] and out["match"].tolist() == [1]
        assert out["sad"].tolist() == [183] and out["residual"].tolist() == [[7 - 190, 0, 0, 0]]
        # one pass: the centres are the corners, (0,0,0) - (4,4,4) moves it onto (4,4,4)
        out = oracle.temporal_predict(ref, rvals, far, np.array([7], np.uint32), 4, L, 0, 1)
        assert out["mv"][0].tolist() == [-4, -4, -4] and out["match"].tolist() == [0]
        lone, _ = oracle.build(np.array([[1, 1, 1]], np.float32), g)
        out = oracle.temporal_predict(lone, np.array([9], np.uint32), far,
                                      np.array([0x01020304], np.uint32), 4, L, 0, 3)
        assert out["mv"][0].tolist() == [-1, -1, -1] and out["match"].tolist() == [0]
        # moved outside the grid: predicted (0,0,0), (7,10,10), (10,10,10)
        # against a reference (0,0,0): cluster 7 settles at (8.5,10,10), motion
        # (9,10,10), so (7,10,10) lands on x = -2: no match, SAD UINT32_MAX, its
        # own channels; (10,10,10) lands on (1,0,0), one step from (0,0,0)
        origin, _ = oracle.build(np.zeros((1, 3), np.float32), g)
        moved, _ = oracle.build(np.array([[0, 0, 0], [7, 10, 10], [10, 10, 10]], np.float32), g)
        out = oracle.temporal_predict(origin, np.array([9], np.uint32), moved,
                                      np.array([9, 0x01020304, 5], np.uint32), 4, L, 2, 9)
        assert out["pred_assign"].tolist() == [0, 7, 7]
        assert out["mv"][7].tolist() == [9, 10, 10] and out["match"].tolist() == [0, -1, 0]
        assert out["sad"].tolist() == [0, 2 ** 32 - 1, 4]
        assert out["residual"].tolist() == [[0, 0, 0, 0], [4, 3, 2, 1], [-4, 0, 0, 0]]
