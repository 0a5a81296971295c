"""Full-size parity, in the launch configuration bench.py times.

One step of bench.py's own pipeline (build two clouds, merge, project onto
XY, k-NN of the queries against the union, learned index of the union and
its lookups next to binary search), in the overlapped form bench.py times,
runs on the GPU at the workloads' full sizes:

* c2: 2 x 1,048,576 LiDAR points, depth 12, 100k queries, k = 8 -- compared
  with the oracle itself (std::map build, std::set_union merge, coordinate
  drop), every one of the 100k k-NN rows with the oracle's kd-tree over the
  whole union, and every lookup with std::lower_bound.
* c2 again on a LINEAR grid: the paper's NN on the five arrays for all 100k
  queries against the kd-tree 1-NN, and its three-level lookup on 200k voxels.
* c6: the temporal-prediction step on the full moving-object frame pair,
  every output against the oracle.
* c4: the 256-frame batch through the captured graph -- every frame's key
  count, and ten frames with their pair unions, against the definitions.
* c5: the 50M-key learned index (linear and network leaves) -- all 10M
  lookups against std::lower_bound.
* c3: 2 x 10M points, depth 14, 1M queries, k = 16 -- build, merge and the
  step's three projections compared with the definitions the oracle states (its
  per-point quantize and key encode, each deduplicated with numpy: a set of
  keys with multiplicities, a set union, the image under a coordinate drop),
  k-NN rows of 4096 queries -- 3584 drawn uniformly from the million and
  the 512 nearest the sphere's centre (those see the whole shell at nearly
  one distance and take the search's most rounds) -- with the oracle's
  kd-tree over the ~20M-voxel union, 32 of them (16 near the centre) also by
  brute force, and a sample of lookups with std::lower_bound.
"""
import numpy as np
import pytest
import torch

import bench
import gen
import oracle
from helpers import say, u64

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _run_step(cga, d, workload):
    pipe = bench.Pipeline(cga, d, torch.device("cuda:0"), bench.WORKLOADS[workload][1])
    pipe.step()
    torch.cuda.synchronize()
    pipe.check()
    pipe.make_lookups()
    pipe.step_concurrent()  # the timed form: independent parts on side streams
    torch.cuda.synchronize()
    pipe.check()
    return pipe


def _keys(t, n):
    return u64(t[:n])


def _check_lookups(pipe, m_ref, sample=None):
    lq = pipe.lq.cpu().numpy().view(np.uint64)
    lrank = pipe.lrank.cpu().numpy()
    brank = pipe.brank.cpu().numpy()
    lfound = pipe.lfound.cpu().numpy()
    if sample is not None:
        lq, lrank, brank, lfound = lq[sample], lrank[sample], brank[sample], lfound[sample]
    want, present = oracle.lower_bound(m_ref, lq)
    np.testing.assert_array_equal(lrank, want)
    np.testing.assert_array_equal(brank, want)
    np.testing.assert_array_equal(lfound.astype(bool), present.astype(bool))


def _check_knn_rows(pipe, rows, idx_ref, d2_ref):
    idx = pipe.idx.cpu().numpy()[rows]
    d2 = pipe.d2.cpu().numpy().view(np.uint64)[rows]
    np.testing.assert_array_equal(idx, idx_ref)
    np.testing.assert_array_equal(d2, d2_ref)


def test_c2_full(gpu):
    cga = gpu
    d = gen.c2_lidar()
    g = d["grid"]
    say("c2 full: build/merge/project/knn/index at 2 x 1048576 points")
    pipe = _run_step(cga, d, "c2")
    ua, ub, um, up = [int(x) for x in pipe.cnt.cpu().tolist()]
    ka, ca = oracle.build(d["a"], g)
    kb, cb = oracle.build(d["b"], g)
    np.testing.assert_array_equal(_keys(pipe.ka, ua), ka)
    np.testing.assert_array_equal(pipe.ca[:ua].cpu().numpy(), ca)
    np.testing.assert_array_equal(_keys(pipe.kb, ub), kb)
    np.testing.assert_array_equal(pipe.cb[:ub].cpu().numpy(), cb)
    m, _ = oracle.merge(ka, kb, g.depth, g.key_mode)
    np.testing.assert_array_equal(_keys(pipe.m, um), m)
    p, pc = oracle.project(m, g.depth, g.key_mode, 2)
    np.testing.assert_array_equal(u64(pipe.p[0][:up]), p)
    np.testing.assert_array_equal(pipe.pc[0][:up].cpu().numpy(), pc)
    # every query row, by the kd-tree over the whole union
    idx_ref, d2_ref = oracle.knn_kdtree(m, d["q"], g, d["k"])
    rows = np.arange(len(d["q"]))
    assert len(rows) == 100_000
    _check_knn_rows(pipe, rows, idx_ref, d2_ref)
    _check_lookups(pipe, m)


def _defined_build(xyz, g):
    keys = oracle.encode(oracle.quantize(xyz, g), g.depth, g.key_mode)
    return np.unique(keys, return_counts=True)


def _defined_project(m, g, drop):
    vox = oracle.decode(m, g.depth, g.key_mode)
    keep = [a for a in range(3) if a != drop]
    pk = oracle.encode2(vox[:, keep[0]], vox[:, keep[1]], g.depth, g.key_mode)
    return np.unique(pk, return_counts=True)


def c3_knn_rows(q, n_uniform=3584, n_centre=512, seed=2003):
    """The k-NN rows checked at full c3 size: a seeded uniform sample of the
    queries plus the n_centre queries nearest the sphere's centre (the
    origin), sorted and distinct."""
    r = np.linalg.norm(q.astype(np.float64), axis=1)
    centre = np.argsort(r, kind="stable")[:n_centre]
    assert r[centre[-1]] < 0.2
    rest = np.setdiff1d(np.arange(len(q)), centre)
    uni = np.random.default_rng(seed).choice(rest, n_uniform, replace=False)
    return np.sort(np.concatenate([centre, uni]))


def test_c3_full(gpu):
    cga = gpu
    d = gen.c3_bumpy()
    g = d["grid"]
    say("c3 full: build/merge/project/knn/index at 2 x 10M points")
    pipe = _run_step(cga, d, "c3")
    cnt = [int(x) for x in pipe.cnt.cpu().tolist()]
    ua, ub, um = cnt[:3]
    assert pipe.drops == (0, 1, 2)
    ka, ca = _defined_build(d["a"], g)
    np.testing.assert_array_equal(_keys(pipe.ka, ua), ka)
    np.testing.assert_array_equal(pipe.ca[:ua].cpu().numpy(), ca)
    kb, cb = _defined_build(d["b"], g)
    np.testing.assert_array_equal(_keys(pipe.kb, ub), kb)
    np.testing.assert_array_equal(pipe.cb[:ub].cpu().numpy(), cb)
    m = np.union1d(ka, kb)
    np.testing.assert_array_equal(_keys(pipe.m, um), m)
    for i, drop in enumerate(pipe.drops):  # the step's three axis projections
        pk, pcnt = _defined_project(m, g, drop)
        up = cnt[3 + i]
        np.testing.assert_array_equal(u64(pipe.p[i][:up]), pk)
        np.testing.assert_array_equal(pipe.pc[i][:up].cpu().numpy(), pcnt)
    rows = c3_knn_rows(d["q"])
    assert len(rows) == 4096
    say("c3 full: kd-tree k-NN of", len(rows), "rows")
    idx_ref, d2_ref = oracle.knn_kdtree(m, d["q"][rows], g, d["k"])
    _check_knn_rows(pipe, rows, idx_ref, d2_ref)
    # a brute-force cross-check of the kd-tree on 32 of them, half near the centre
    near = rows[np.linalg.norm(d["q"][rows].astype(np.float64), axis=1) < 0.2]
    assert len(near) >= 16
    sub = np.sort(np.concatenate([near[:16], rows[~np.isin(rows, near)][::224][:16]]))
    say("c3 full: brute-force k-NN of", len(sub), "rows")
    idx_b, d2_b = oracle.knn_brute(m, d["q"][sub], g, d["k"])
    _check_knn_rows(pipe, sub, idx_b, d2_b)
    _check_lookups(pipe, m, sample=np.arange(0, len(pipe.lq), 7))


def test_c2_paper_array_ops_full(gpu):
    """The paper's lookup and NN on the five arrays of the full c2 union
    (LINEAR): every NN row vs the kd-tree 1-NN, lookups vs the oracle's
    three-level search on 200k voxels."""
    cga = gpu
    d = gen.c2_lidar()
    g = d["grid"].with_mode(gen.KEY_LINEAR)
    ka, _ = oracle.build(d["a"], g)
    kb, _ = oracle.build(d["b"], g)
    m, _ = oracle.merge(ka, kb, g.depth, g.key_mode)
    say("c2 paper array ops: union", len(m))
    mk = cga.cga_build(torch.from_numpy(d["a"]).to("cuda:0"), g)[0]
    mb = cga.cga_build(torch.from_numpy(d["b"]).to("cuda:0"), g)[0]
    mg, _ = cga.cga_merge(mk, mb, g)
    arr = cga.cga_to_arrays(mg, g)
    idx, d2 = cga.cga_arrays_nn(arr, torch.from_numpy(d["q"]).to("cuda:0"), g)
    widx, wd2 = oracle.knn_kdtree(m, d["q"], g, 1)
    np.testing.assert_array_equal(d2.cpu().numpy().view(np.uint64), wd2[:, 0])
    np.testing.assert_array_equal(idx.cpu().numpy(), widx[:, 0])
    rng = np.random.default_rng(2004)
    qv = np.concatenate([oracle.decode(m[rng.integers(0, len(m), 100_000)], g.depth, g.key_mode),
                         rng.integers(0, 2 ** g.depth, (100_000, 3))]).astype(np.uint32)
    pos = cga.cga_arrays_lookup(arr, torch.from_numpy(qv.view(np.int32)).to("cuda:0"), g)
    np.testing.assert_array_equal(pos.cpu().numpy(), oracle.lookup_cga(oracle.arrays(m, g.depth, g.key_mode), qv))


def test_c6_temporal_full(gpu):
    """The temporal step on the full moving-object frame pair (1024^3 grid),
    in the configuration bench.py times (window 2, at most 100 passes):
    every output vs the oracle."""
    cga = gpu
    d = gen.c6_frames()
    g = d["grid"]
    ref, rv = oracle.voxel_values(d["ref"], d["ref_values"], g)
    pred, pv = oracle.voxel_values(d["pred"], d["pred_values"], g)
    say("c6 temporal full:", len(ref), len(pred))
    want = oracle.temporal_predict(ref, rv, pred, pv, g.depth, g.key_mode, 2, 100)
    dev = torch.device("cuda:0")
    got = cga.cga_temporal_predict(torch.from_numpy(ref.astype(np.uint32).view(np.int32)).to(dev),
                                   torch.from_numpy(rv.view(np.int32)).to(dev),
                                   torch.from_numpy(pred.astype(np.uint32).view(np.int32)).to(dev),
                                   torch.from_numpy(pv.view(np.int32)).to(dev), g, window=2,
                                   max_iter=100)
    for name in ("ref_assign", "pred_assign", "centroids", "mv", "iters", "match", "residual"):
        np.testing.assert_array_equal(got[name].cpu().numpy(), want[name], err_msg=name)
    np.testing.assert_array_equal(got["sad"].cpu().numpy().view(np.uint32), want["sad"])


def test_c4_full(gpu):
    """The 256-frame batch (92.6M points) through the captured graph, as bench.py
    replays it: ten frames and their pair unions against the definitions
    (per-point quantize and key encode, np.unique, np.union1d), and every
    frame's key count against one np.unique over (frame, key)."""
    cga = gpu
    d = gen.c4_frames()
    g, xyz, off = d["grid"], d["xyz"], d["off"]
    F = len(off) - 1
    say("c4 full:", F, "frames,", len(xyz), "points")
    dev = torch.device("cuda:0")
    graph = cga.BatchGraph(torch.from_numpy(xyz).to(dev), torch.from_numpy(off).to(dev), g)
    graph.launch()
    torch.cuda.synchronize()
    assert graph.status() == 0
    keys = oracle.encode(oracle.quantize(xyz, g), g.depth, g.key_mode)
    frame = np.repeat(np.arange(F, dtype=np.uint64), np.diff(off))
    comp = np.unique((frame << np.uint64(3 * g.depth)) | keys)
    per_frame = np.bincount((comp >> np.uint64(3 * g.depth)).astype(np.int64), minlength=F)
    np.testing.assert_array_equal(np.diff(graph.out.key_off.cpu().numpy()), per_frame)
    rng = np.random.default_rng(2005)
    picks = sorted(set([0, 1, F - 2] + rng.choice(F - 1, 7, replace=False).tolist()))
    for f in picks:
        kf = np.unique(keys[off[f]:off[f + 1]])
        kn = np.unique(keys[off[f + 1]:off[f + 2]])
        np.testing.assert_array_equal(_keys(graph.out.frame(f), len(kf)), kf)
        np.testing.assert_array_equal(u64(graph.out.pair(f)), np.union1d(kf, kn))
    graph.close()


def test_c5_full(gpu):
    """The 50M-key learned index as bench.py trains it (linear leaves, 65,536
    leaves, 4096-segment root; and 65,536 network leaves), keys built by the
    definition (quantize, encode, np.unique, the seeded subset), all 10M
    lookups against the oracle's std::lower_bound."""
    cga = gpu
    d = gen.c5_sweeps()
    g = d["grid"]
    keys = np.unique(oracle.encode(oracle.quantize(d["xyz"], g), g.depth, g.key_mode))
    del d
    u, target = len(keys), 50_000_000
    if u > target:
        keys = keys[gen.subset(1005, u, target)]
    q = gen.lookup_queries(1005, keys, 10_000_000)
    say("c5 full:", len(keys), "keys,", len(q), "lookups")
    rank_want, found_want = oracle.lower_bound(keys, q)
    dev = torch.device("cuda:0")
    kd = torch.from_numpy(keys.view(np.int64)).to(dev)
    qd = torch.from_numpy(q.view(np.int64)).to(dev)
    for kind, leaves, root in ((0, 65536, 4096), (cga.LEAF_MLP, 65536, 4096), (0, 1 << 24, 4096),
                               (cga.LEAF_MLP, 1 << 18, 4096)):
        idx = cga.cga_index_train(kd, n_leaves=leaves, leaf_kind=kind, root_segments=root)
        r, f, _ = cga.cga_index_lookup(idx, kd, qd)
        np.testing.assert_array_equal(r.cpu().numpy(), rank_want)
        np.testing.assert_array_equal(f.cpu().numpy().astype(bool), found_want.astype(bool))
    r, f = cga.cga_binary_lookup(kd, qd)
    np.testing.assert_array_equal(r.cpu().numpy(), rank_want)
