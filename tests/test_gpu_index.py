"""GPU tests of the learned index: exact ranks against the oracle's
lower_bound on every query (present, absent, extremes), the binary-search
fallback when the windows are wrong, key-array mismatch detection, the leaf
network's gradient against the fp64 oracle, and what the trained network
gains over linear leaves and over no index."""
import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import dev, say

pytestmark = pytest.mark.gpu


def _lidar_keys(nsweeps=4, naz=4096, depth=16):
    """Sorted unique 48-bit Morton keys of a few LiDAR sweeps (oracle build)."""
    boxes = gen.lidar_scene(1005)
    poses, _ = gen.random_walk(1005, nsweeps)
    xyz = np.concatenate([gen.lidar_sweep(1005, 100 + f, boxes, poses[f, :3], poses[f, 3], 64, naz)
                          for f in range(nsweeps)])
    g = gen.cubic_grid([xyz], depth)
    keys, _ = oracle.build(xyz, g)
    return keys


@pytest.fixture(scope="module")
def lidar_keys():
    return _lidar_keys()


def _queries(keys, nq, seed):
    q = gen.lookup_queries(seed, keys, nq)
    extra = np.array([0, 2 ** 64 - 1, keys[0], keys[-1], keys[0] - 1, keys[-1] + 1,
                      keys[len(keys) // 2] + 1], np.uint64)
    return np.concatenate([q, extra])


def _t(a):
    return dev(np.ascontiguousarray(a, np.uint64).view(np.int64))


@pytest.mark.parametrize("kind,leaves,root", [(0, 4096, 0), (1, 4096, 0), (0, 4096, 1024),
                                              (1, 4096, 1024), (1, 1, 0), (0, 7, 3), (1, 65536, 64),
                                              (1, 4096, 65536), (0, 1 << 20, 4096),
                                              (0, 1 << 24, 65536), (1, 1 << 18, 4096),
                                              (0, 1 << 16, 4097), (0, 1 << 16, 5000)])
def test_lookup_exact(gpu, lidar_keys, kind, leaves, root):
    keys = lidar_keys
    q = _queries(keys, 200_000, 7 + kind)
    kd, qd = _t(keys), _t(q)
    say("index", kind, leaves, root, len(keys))
    idx = gpu.cga_index_train(kd, n_leaves=leaves, leaf_kind=kind, epochs=20, root_segments=root)
    r, f, fb = gpu.cga_index_lookup(idx, kd, qd)
    wr, wf = oracle.lower_bound(keys, q)
    assert np.array_equal(r.cpu().numpy(), wr)
    assert np.array_equal(f.cpu().numpy(), wf)
    br, bf = gpu.cga_binary_lookup(kd, qd)
    assert np.array_equal(br.cpu().numpy(), wr) and np.array_equal(bf.cpu().numpy(), wf)
    # present keys never fall back: their windows are measured on them
    rp, _, fbp = gpu.cga_index_lookup(idx, kd, kd)
    assert fbp == 0 and np.array_equal(rp.cpu().numpy(), np.arange(len(keys)))


def test_lookup_small_arrays(gpu):
    for keys in (np.array([5], np.uint64), np.array([1, 2], np.uint64),
                 np.unique(np.random.default_rng(1).integers(0, 2 ** 40, 3000, dtype=np.uint64))):
        q = np.concatenate([keys, keys + np.uint64(1), np.array([0, 2 ** 64 - 1], np.uint64)])
        for kind, root in ((0, 0), (1, 0), (0, 16), (1, 1024)):
            kd = _t(keys)
            idx = gpu.cga_index_train(kd, n_leaves=64, leaf_kind=kind, epochs=5, root_segments=root)
            r, f, _ = gpu.cga_index_lookup(idx, kd, _t(q))
            wr, wf = oracle.lower_bound(keys, q)
            assert np.array_equal(r.cpu().numpy(), wr) and np.array_equal(f.cpu().numpy(), wf)


def _window_offsets(n_leaves, nparams, root):
    """Byte offsets of every leaf's err_lo / err_hi in the index buffer: a
    256-byte header, the root segment starts (8 B each) and segments (32 B
    each), the 4096-key fingerprint (8 B each), then one record per leaf (64 B
    for linear leaves, 256 B for network leaves) whose window sits at bytes
    24 and 28."""
    al = lambda v: (v + 255) // 256 * 256
    off = al(256 + root * 8)
    off = al(off + root * 32)
    off = al(off + 4096 * 8)
    stride = 64 if nparams <= 8 else 256
    base = off + np.arange(n_leaves) * stride
    return base + 24, base + 28


def test_zeroed_windows_fall_back_and_stay_exact(gpu, lidar_keys):
    keys = lidar_keys
    kd = _t(keys)
    idx = gpu.cga_index_train(kd, n_leaves=4096, leaf_kind=1, epochs=10, root_segments=1024)
    host = idx.cpu().numpy().copy()
    lo, hi = _window_offsets(4096, 49, 1024)
    # the offsets land on the leaf records: their key counts (bytes 16..19)
    # are the index's own, and each leaf's window was ordered
    i32 = lambda offs: np.array([int(np.frombuffer(host[o:o + 4].tobytes(), np.int32)[0])
                                 for o in offs])
    _, cnt = gpu.cga_index_stats(idx, 4096)
    assert np.array_equal(i32(lo - 8), cnt.cpu().numpy())
    full = cnt.cpu().numpy() > 0
    assert (i32(lo)[full] <= i32(hi)[full]).all()
    for off in np.concatenate([lo, hi]):
        host[off:off + 4] = 0
    bad = torch.from_numpy(host).cuda()
    q = _queries(keys, 100_000, 11)
    r, f, fb = gpu.cga_index_lookup(bad, kd, _t(q))
    wr, wf = oracle.lower_bound(keys, q)
    assert np.array_equal(r.cpu().numpy(), wr) and np.array_equal(f.cpu().numpy(), wf)
    assert fb > 0


def test_mismatched_keys_rejected(gpu, lidar_keys):
    keys = lidar_keys
    idx = gpu.cga_index_train(_t(keys), n_leaves=256, leaf_kind=0)
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_index_lookup(idx, _t(keys[:-1]), _t(keys[:10]))
    assert e.value.status == gpu.EMISMATCH


def _same_ends(keys, seed):
    """Another sorted unique array with the same size and the same first and
    last keys: every interior key redrawn uniformly between them."""
    rng = np.random.default_rng(seed)
    inner = np.unique(rng.integers(keys[0] + np.uint64(1), keys[-1], 2 * len(keys), dtype=np.uint64))
    inner = np.sort(rng.choice(inner, len(keys) - 2, replace=False))
    out = np.concatenate([keys[:1], inner, keys[-1:]])
    assert len(out) == len(keys) and (np.diff(out) > 0).all()
    return out


@pytest.mark.parametrize("kind,leaves,root", [(0, 4096, 0), (1, 4096, 1024), (0, 1 << 20, 4096)])
def test_same_size_same_ends_other_keys(gpu, lidar_keys, kind, leaves, root):
    """An array with the index's n, first and last key but other interior
    keys: the lookup reports CGA_EMISMATCH (the fingerprint ranks differ),
    and its ranks are still the exact lower bounds in that array (every
    window is verified against the array it searches)."""
    keys = lidar_keys
    other = _same_ends(keys, 31 + kind)
    idx = gpu.cga_index_train(_t(keys), n_leaves=leaves, leaf_kind=kind, epochs=10,
                              root_segments=root)
    q = _queries(other, 100_000, 13)
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_index_lookup(idx, _t(other), _t(q))
    assert e.value.status == gpu.EMISMATCH
    ws = gpu.Workspaces()
    r, f, fb = gpu.cga_index_lookup(idx, _t(other), _t(q), sync=False, ws=ws)
    torch.cuda.synchronize()
    wr, wf = oracle.lower_bound(other, q)
    assert np.array_equal(r.cpu().numpy(), wr) and np.array_equal(f.cpu().numpy(), wf)
    assert int(fb.item()) > 0
    # one interior key changed at a sampled rank is caught as well
    one = keys.copy()
    mid = (2048 * (len(keys) - 1)) // 4095
    assert keys[mid - 1] + np.uint64(1) < keys[mid]
    one[mid] = keys[mid] - np.uint64(1)
    with pytest.raises(gpu.CgaError) as e:
        gpu.cga_index_lookup(idx, _t(one), _t(q))
    assert e.value.status == gpu.EMISMATCH
    # the trained array itself passes
    r, f, _ = gpu.cga_index_lookup(idx, _t(keys), _t(q))
    wr, wf = oracle.lower_bound(keys, q)
    assert np.array_equal(r.cpu().numpy(), wr) and np.array_equal(f.cpu().numpy(), wf)


def test_mlp_gradient_matches_fp64_oracle(gpu):
    rng = np.random.default_rng(3)
    for n in (1, 37, 1000, 20000):
        p = rng.normal(0, 1, 49).astype(np.float32)
        x = np.sort(rng.uniform(0, 1, n)).astype(np.float32)
        t = np.sort(rng.uniform(0, 1, n)).astype(np.float32)
        loss, g = gpu.cga_mlp_loss_grad(dev(p), dev(x), dev(t))
        wl, wg, kinks = oracle.mlp_loss_grad(p.astype(np.float64), x.astype(np.float64),
                                             t.astype(np.float64))
        assert kinks == 0
        g = g.cpu().numpy()
        scale = max(1.0, np.abs(wg).max())
        assert np.allclose(g, wg, rtol=1e-4, atol=1e-5 * scale), (n, np.abs(g - wg).max())
        assert abs(loss - wl) <= 1e-4 * max(1.0, wl)


def test_mlp_gradient_edges(gpu):
    """Repeated x values, a unit active everywhere / nowhere / on a run that
    ascends or descends, and x that does not ascend (NaN outputs)."""
    rng = np.random.default_rng(4)
    p = rng.normal(0, 1, 49).astype(np.float32)
    p[0], p[16] = 0.0, 0.5    # w1 = 0, b1 > 0: active on every sample
    p[1], p[17] = 0.0, -0.5   # w1 = 0, b1 < 0: never active
    p[2], p[18] = -3.0, 1.505  # descending: active below x = 0.5017
    p[3], p[19] = 2.0, -0.25  # ascending: active above x = 0.125
    x = np.sort(np.round(rng.uniform(0, 1, 700), 2)).astype(np.float32)  # many repeats
    t = np.sort(rng.uniform(0, 1, 700)).astype(np.float32)
    loss, g = gpu.cga_mlp_loss_grad(dev(p), dev(x), dev(t))
    wl, wg, kinks = oracle.mlp_loss_grad(p.astype(np.float64), x.astype(np.float64),
                                         t.astype(np.float64))
    assert kinks == 0
    g = g.cpu().numpy()
    assert np.allclose(g, wg, rtol=1e-4, atol=1e-5 * max(1.0, np.abs(wg).max()))
    assert abs(loss - wl) <= 1e-4 * max(1.0, wl)
    xb = x.copy()
    xb[[10, 11]] = xb[[11, 10]] if xb[10] != xb[11] else (xb[10], xb[10] - 0.5)
    loss, g = gpu.cga_mlp_loss_grad(dev(p), dev(xb), dev(t))
    assert np.isnan(loss) and np.isnan(g.cpu().numpy()).all()


def test_trained_network_gain(gpu, lidar_keys):
    """Mean window width and fallback rate: linear leaves, the network at its
    initialisation, and the trained network; plus the binary-search probe
    count for the same array.  The trained network must not be worse than its
    initialisation and must beat linear leaves."""
    keys = lidar_keys
    kd = _t(keys)
    q = _queries(keys, 200_000, 13)
    qd = _t(q)
    wr, _ = oracle.lower_bound(keys, q)
    res = {}
    for name, kind, ep, root in (("linear_root+linear", 0, 0, 0), ("linear_root+mlp", 1, 200, 0),
                                 ("linear", 0, 0, 1024), ("mlp_init", 1, 0, 1024),
                                 ("mlp_trained", 1, 200, 1024)):
        idx = gpu.cga_index_train(kd, n_leaves=4096, leaf_kind=kind, epochs=ep, lr=1e-4,
                                  root_segments=root)
        w, c = gpu.cga_index_stats(idx, 4096)
        w, c = w.cpu().numpy().astype(np.float64), c.cpu().numpy()
        mean_w = float((w * c).sum() / c.sum())
        r, _, fb = gpu.cga_index_lookup(idx, kd, qd)
        assert np.array_equal(r.cpu().numpy(), wr)
        res[name] = (mean_w, fb / len(q))
    say("window width (key-weighted mean) / fallback rate:", res,
        "binary search probes:", int(np.ceil(np.log2(len(keys)))))
    assert res["mlp_trained"][0] <= res["mlp_init"][0] * 1.001
    assert res["mlp_trained"][0] < res["linear"][0]
