#!/usr/bin/env python3
"""Benchmark of the CGA hot path on one MI355X.

One step = the whole pipeline on one batch of synthetic input, already in
HBM: build the CGA of two LiDAR sweeps (quantize, encode, radix sort,
run-length compaction), merge them, project the union onto XY, answer k-NN
queries against the union, train the learned index of the union and answer
point-location / range-start lookups with it and with binary search.
Workloads:
  c2 (default): 2 x 1,048,576-point sweeps, depth 12, 100k queries, k = 8
  c3: 2 x 10M-point bumpy spheres, depth 14, 1M queries, k = 16
  c1: 2 x 100k sphere points, depth 10, 1k queries, k = 1
Prints one JSON line.  value = input points per second of whole steps.
Unless --no-c5, it also measures the learned index against binary search on
the 50M-key, 10M-query configuration (reported under "c5"), and unless
--no-c4 the graph-captured batched build + pair merge of 256 LiDAR frames
(reported under "c4"); neither enters value.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the per-kernel event timing (for external profilers)")
    ap.add_argument("--no-c5", action="store_true", help="skip the 50M-key learned-index run")
    ap.add_argument("--c5-reps", type=int, default=10)
    ap.add_argument("--no-c4", action="store_true", help="skip the 256-frame batched run")
    ap.add_argument("--c4-reps", type=int, default=5)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers 5 times (a plain copy "
                         "kernel of known size, to scale hardware byte counters)")
    return ap.parse_args()


def copy_calibration(nbytes):
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                      "reps": 5}))


def make_workload(name):
    import gen
    if name == "c1":
        d = gen.c1_spheres()
    elif name == "c3":
        d = gen.c3_bumpy()
    else:
        d = gen.c2_lidar()
    return d


class Pipeline:
    """Preallocated buffers and workspaces for one step; every size stays on
    the device between calls."""

    def __init__(self, cga, d, device):
        import torch
        self.cga, self.g, self.k = cga, d["grid"], d["k"]
        self.a = torch.from_numpy(d["a"]).to(device)
        self.b = torch.from_numpy(d["b"]).to(device)
        self.q = torch.from_numpy(d["q"]).to(device)
        na, nb = len(self.a), len(self.b)
        kt, k2t = cga.key_dtype(self.g), cga.key2_dtype(self.g)
        self.na, self.nb, self.nm = na, nb, na + nb
        e = lambda n, t: torch.empty(max(n, 1), dtype=t, device=device)
        self.ka, self.ca = e(na, kt), e(na, torch.int32)
        self.kb, self.cb = e(nb, kt), e(nb, torch.int32)
        self.m = e(self.nm, kt)
        self.p, self.pc = e(self.nm, k2t), e(self.nm, torch.int32)
        nq = len(self.q)
        self.idx = torch.empty((nq, self.k), dtype=torch.int64, device=device)
        self.d2 = torch.empty((nq, self.k), dtype=torch.int64, device=device)
        self.cnt = torch.zeros(4, dtype=torch.int64, device=device)
        self.ws = [cga.Workspaces(device) for _ in range(7)]
        # learned index of the union: a buffer sized for it, and lookups of
        # the union's own keys (half) and uniform values (half); the present
        # half is drawn by position from the oracle-independent generator on
        # the host after one synchronous build (setup, outside the timing)
        self.index_kwargs = dict(n_leaves=4096, leaf_kind=cga.LEAF_MLP, epochs=50, lr=1e-4,
                                 root_segments=1024)
        p = cga.index_params(**self.index_kwargs)
        self.index = torch.empty(cga.lib.cga_index_bytes(ctypes.byref(p)), dtype=torch.uint8,
                                 device=device)
        self.nl = 100_000
        self.lq = None
        self.lrank = torch.empty(self.nl, dtype=torch.int64, device=device)
        self.lfound = torch.empty(self.nl, dtype=torch.uint8, device=device)
        self.brank = torch.empty(self.nl, dtype=torch.int64, device=device)
        self.bfound = torch.empty(self.nl, dtype=torch.uint8, device=device)
        self.fb = torch.zeros(1, dtype=torch.int64, device=device)
        # side streams (default priority) for the independent parts of a step
        self.side = [torch.cuda.Stream(device=device) for _ in range(4)]
        self.ev = [torch.cuda.Event() for _ in range(6)]

    def make_lookups(self, seed=1006):
        import numpy as np
        import torch

        import gen
        m = self.m[: int(self.cnt[2].item())].cpu().numpy().view(np.uint64)
        self.lq = torch.from_numpy(gen.lookup_queries(seed, m, self.nl).view(np.int64)).to(
            self.m.device)

    def step(self, marks=None):
        c, g = self.cga, self.g
        cnt = self.cnt
        if marks:
            marks[0].record()
        c.cga_build(self.a, g, keys_out=self.ka, counts_out=self.ca, d_n_out=cnt[0:1], sync=False,
                    ws=self.ws[0])
        c.cga_build(self.b, g, keys_out=self.kb, counts_out=self.cb, d_n_out=cnt[1:2], sync=False,
                    ws=self.ws[1])
        c.cga_merge(self.ka, self.kb, g, na=self.na, d_na=cnt[0:1], nb=self.nb, d_nb=cnt[1:2],
                    out=self.m, d_n_out=cnt[2:3], sync=False, ws=self.ws[2])
        if marks:
            marks[1].record()
        c.cga_project(self.m, g, 2, n=self.nm, d_n=cnt[2:3], out=self.p, counts_out=self.pc,
                      d_n_out=cnt[3:4], sync=False, ws=self.ws[3])
        if marks:
            marks[2].record()
        c.cga_knn(self.m, self.q, g, self.k, n=self.nm, d_n=cnt[2:3], idx_out=self.idx,
                  d2_out=self.d2, sync=False, ws=self.ws[4])
        if marks:
            marks[3].record()
        if self.lq is not None:
            # the index is trained on the union; its size comes from the host
            # copy taken at setup (the merge result is identical every step)
            c.cga_index_train(self.m, self.nu, out=self.index, ws=self.ws[5], **self.index_kwargs)
            if marks:
                marks[4].record()
            c.cga_index_lookup(self.index, self.m, self.lq, n=self.nu, rank_out=self.lrank,
                               found_out=self.lfound, fallbacks_out=self.fb, sync=False,
                               ws=self.ws[6])
            if marks:
                marks[5].record()
            c.cga_binary_lookup(self.m, self.lq, n=self.nu, rank_out=self.brank,
                                found_out=self.bfound)
            if marks:
                marks[6].record()

    def step_concurrent(self):
        """The same step with its independent parts overlapped on side
        streams: the two builds side by side, then the merge, then the
        projection, the k-NN search and the index training + lookups side by
        side; the step ends when all have (the next step's builds overwrite
        what they read)."""
        import torch
        c, g, cnt = self.cga, self.g, self.cnt
        main = torch.cuda.current_stream()
        sb, sp, sk, si = self.side
        ev = self.ev
        ev[0].record(main)
        sb.wait_event(ev[0])
        c.cga_build(self.a, g, keys_out=self.ka, counts_out=self.ca, d_n_out=cnt[0:1], sync=False,
                    ws=self.ws[0])
        with torch.cuda.stream(sb):
            c.cga_build(self.b, g, keys_out=self.kb, counts_out=self.cb, d_n_out=cnt[1:2],
                        sync=False, ws=self.ws[1])
        ev[1].record(sb)
        main.wait_event(ev[1])
        c.cga_merge(self.ka, self.kb, g, na=self.na, d_na=cnt[0:1], nb=self.nb, d_nb=cnt[1:2],
                    out=self.m, d_n_out=cnt[2:3], sync=False, ws=self.ws[2])
        ev[2].record(main)
        for s in (sp, sk, si):
            s.wait_event(ev[2])
        # the k-NN search, the longest branch, is issued first
        with torch.cuda.stream(sk):
            c.cga_knn(self.m, self.q, g, self.k, n=self.nm, d_n=cnt[2:3], idx_out=self.idx,
                      d2_out=self.d2, sync=False, ws=self.ws[4])
        with torch.cuda.stream(sp):
            c.cga_project(self.m, g, 2, n=self.nm, d_n=cnt[2:3], out=self.p, counts_out=self.pc,
                          d_n_out=cnt[3:4], sync=False, ws=self.ws[3])
        with torch.cuda.stream(si):
            c.cga_index_train(self.m, self.nu, out=self.index, ws=self.ws[5], **self.index_kwargs)
            c.cga_index_lookup(self.index, self.m, self.lq, n=self.nu, rank_out=self.lrank,
                               found_out=self.lfound, fallbacks_out=self.fb, sync=False,
                               ws=self.ws[6])
            c.cga_binary_lookup(self.m, self.lq, n=self.nu, rank_out=self.brank,
                                found_out=self.bfound)
        for e, s in zip(ev[3:6], (sp, sk, si)):
            e.record(s)
            main.wait_event(e)

    def check(self):
        for w in self.ws:
            for buf in w.bufs.values():
                st = self.cga.lib.cga_ws_status(self.cga._ptr(buf), self.cga._stream())
                if st != 0:
                    raise self.cga.CgaError(st, "bench step")


def step_outputs(pipe):
    """Copies of everything one step writes (the arrays up to their counts)."""
    ua, ub, um, up = pipe.cnt.tolist()
    return [t.clone() for t in (pipe.cnt, pipe.ka[:ua], pipe.kb[:ub], pipe.m[:um], pipe.p[:up],
                                pipe.pc[:up], pipe.idx, pipe.d2, pipe.index, pipe.lrank,
                                pipe.lfound, pipe.brank, pipe.bfound)]


def graph_step(pipe, steps):
    """The overlapped step captured once into a HIP graph (its side streams
    become branches of the graph) and replayed: the same kernels, launched
    without per-kernel host work.  Every output of the first replay and of
    the last timed one must equal an eager step's, with eager steps and
    synchronisations in between.  Returns ms per replayed step."""
    import torch
    pipe.step_concurrent()
    torch.cuda.synchronize()
    want = step_outputs(pipe)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=cap):
        pipe.step_concurrent()
    torch.cuda.synchronize()

    def same():
        got = step_outputs(pipe)
        return all(torch.equal(a, b) for a, b in zip(got, want))

    graph.replay()
    torch.cuda.synchronize()
    if not same():
        raise RuntimeError("graph replay of the step differs from the eager step")
    pipe.step_concurrent()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        graph.replay()
    stop.record()
    torch.cuda.synchronize()
    pipe.check()
    if not same():
        raise RuntimeError("graph replay of the step differs from the eager step")
    return start.elapsed_time(stop) / steps


def algorithmic_bytes(label, pipe, counts):
    """Bytes the method itself must move in one step for a kernel label
    (reads + writes of its essential inputs and outputs)."""
    kb = 8 if 3 * pipe.g.depth > 32 else 4
    k2b = 8 if 2 * pipe.g.depth > 32 else 4
    rb = 8
    passes3 = -(-3 * pipe.g.depth // rb)
    passes2 = -(-2 * pipe.g.depth // rb)
    ua, ub, um, up = counts
    if label == "onesweep":
        # every pass reads and writes each key once
        return passes3 * 2 * kb * (pipe.na + pipe.nb) + passes2 * 2 * k2b * um
    if label == "encode":
        return (12 + kb) * (pipe.na + pipe.nb)
    if label == "rle":
        return kb * (pipe.na + pipe.nb) + (kb + 4) * (ua + ub) + k2b * um + (k2b + 4) * up
    if label == "merge":
        return kb * (ua + ub + um)
    if label == "rekey":
        return (kb + k2b) * um
    if label == "knn_tree":
        # read every key of the union once
        return kb * um
    if label == "knn":
        # per query: read the query (12 B), write k (index, d2) pairs (16 B
        # each), read at least the k result keys
        nq = len(pipe.q)
        return nq * (12 + 16 * pipe.k + kb * pipe.k)
    return None


def kernel_source_sha():
    import glob
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2110_11616_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def load_traffic(label, workload):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a plain
    copy of known size), or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{label}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(d, lookups=None):
    """The oracle, untuned, on one full step of the same workload (the
    learned index has no oracle counterpart beyond lower_bound itself)."""
    import numpy as np

    import oracle
    g = d["grid"]
    t_set = t_knn = 0.0
    steps = 0
    # whole steps, repeated until about 10 s of CPU work (at least one)
    while steps == 0 or (t_set + t_knn < 10.0 and steps < 50):
        t0 = time.perf_counter()
        ka, _ = oracle.build(d["a"], g)
        kb, _ = oracle.build(d["b"], g)
        m, _ = oracle.merge(ka, kb, g.depth, g.key_mode)
        oracle.project(m, g.depth, g.key_mode, 2)
        t1 = time.perf_counter()
        oracle.knn_kdtree(m, d["q"], g, d["k"])
        if lookups is not None:
            oracle.lower_bound(m, lookups)
        t2 = time.perf_counter()
        t_set += t1 - t0
        t_knn += t2 - t1
        steps += 1
    n = len(d["a"]) + len(d["b"])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    per = (t_set + t_knn) / steps
    return {
        "value": n / per, "unit": "points/s", "cores": threads, "kind": "oracle",
        "sample": (f"{steps} full step(s) of {n} points and {len(d['q'])} queries: std::map/std::set "
                   f"build, merge and projection on 1 thread ({t_set / steps:.2f} s/step), kd-tree "
                   f"k-NN and lower_bound lookups on {threads} OpenMP threads "
                   f"({t_knn / steps:.2f} s/step)"),
        "seconds_per_step": round(per, 3),
    }


C5_VARIANTS = (("linear_leaves_16777216_pl4096", 0, 1 << 24, 4096),
               ("linear_leaves_4194304_pl4096", 0, 1 << 22, 4096),
               ("linear_leaves_1048576_pl4096", 0, 1 << 20, 4096),
               ("linear_leaves_65536_pl4096", 0, 65536, 4096),
               ("mlp_leaves_262144_pl4096", 1, 1 << 18, 4096),
               ("mlp_leaves_65536_pl4096", 1, 65536, 4096),
               ("mlp_leaves_4096_pl1024", 1, 4096, 1024))


def c5_learned_vs_binary(cga, device, reps, variants=C5_VARIANTS):
    """The 50M-key configuration: build the keys of random-walk LiDAR sweeps at
    depth 16, keep a seeded uniform subset of exactly 50M, train the index,
    then time 10M lookups (half present, half uniform in the key range) with
    the learned index and with binary search, interleaved on one stream, and
    require identical ranks and membership."""
    import numpy as np
    import torch

    import gen
    t0 = time.perf_counter()
    d = gen.c5_sweeps()
    xyz = torch.from_numpy(d["xyz"]).to(device)
    keys, _ = cga.cga_build(xyz, d["grid"], counts=False)
    del xyz
    u = len(keys)
    target = 50_000_000
    if u > target:
        sel = torch.from_numpy(gen.subset(1005, u, target)).to(device)
        keys = keys.index_select(0, sel).contiguous()
    n = len(keys)
    kh = keys.cpu().numpy().view(np.uint64)
    q = torch.from_numpy(gen.lookup_queries(1005, kh, 10_000_000).view(np.int64)).to(device)
    setup_s = time.perf_counter() - t0
    out = {"keys": n, "unique_before_subset": u, "queries": len(q), "setup_s": round(setup_s, 1)}
    res = {}
    for name, kind, leaves, root in variants:
        torch.cuda.synchronize()
        a = time.perf_counter()
        idx = cga.cga_index_train(keys, n_leaves=leaves, leaf_kind=kind, epochs=50, lr=1e-4,
                                  root_segments=root)
        torch.cuda.synchronize()
        train_ms = (time.perf_counter() - a) * 1e3
        w, c = cga.cga_index_stats(idx, leaves)
        w, c = w.cpu().numpy().astype(np.float64), c.cpu().numpy()
        res[name] = {"train_ms": round(train_ms, 2),
                     "window_mean": round(float((w * c).sum() / max(c.sum(), 1)), 2),
                     "idx": idx}
    rank_l = torch.empty(len(q), dtype=torch.int64, device=device)
    found_l = torch.empty(len(q), dtype=torch.uint8, device=device)
    rank_b = torch.empty_like(rank_l)
    found_b = torch.empty_like(found_l)
    fb = torch.zeros(1, dtype=torch.int64, device=device)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    times = {k: [] for k in list(res) + ["binary"]}
    for _ in range(reps):
        for name in res:
            e0, e1 = ev(), ev()
            e0.record()
            cga.cga_index_lookup(res[name]["idx"], keys, q, rank_out=rank_l, found_out=found_l,
                                 fallbacks_out=fb, sync=False)
            e1.record()
            times[name].append((e0, e1))
        e0, e1 = ev(), ev()
        e0.record()
        cga.cga_binary_lookup(keys, q, rank_out=rank_b, found_out=found_b)
        e1.record()
        times["binary"].append((e0, e1))
    torch.cuda.synchronize()
    med = lambda xs: float(np.median([a.elapsed_time(b) for a, b in xs]))
    for name in res:
        fb.zero_()
        r, f, nfb = cga.cga_index_lookup(res[name]["idx"], keys, q, rank_out=rank_l, found_out=found_l,
                                        fallbacks_out=fb)
        cga.cga_binary_lookup(keys, q, rank_out=rank_b, found_out=found_b)
        torch.cuda.synchronize()
        same = bool(torch.equal(rank_l, rank_b) and torch.equal(found_l, found_b))
        if not same:
            raise RuntimeError(f"learned lookup ({name}) disagrees with binary search")
        ms = med(times[name])
        del res[name]["idx"]
        res[name].update({"lookup_ms": round(ms, 3), "lookups_per_s": len(q) / (ms * 1e-3),
                          "fallback_rate": nfb / len(q), "identical_to_binary": same})
    ms_b = med(times["binary"])
    out["binary"] = {"lookup_ms": round(ms_b, 3), "lookups_per_s": len(q) / (ms_b * 1e-3)}
    out["learned"] = res
    out["speedup_best_learned_vs_binary"] = round(
        max(v["lookups_per_s"] for v in res.values()) / out["binary"]["lookups_per_s"], 3)
    return out


def occupancy_codes(cga, pipe, reps=20):
    """Octree occupancy codes of the step's union (not part of the step):
    average time of one cga_occupancy call, device sizes, events around reps."""
    import torch
    n = pipe.nu
    occ = torch.empty(cga.occupancy_bound(n, pipe.g.depth), dtype=torch.uint8, device=pipe.m.device)
    counts = torch.empty(pipe.g.depth + 1, dtype=torch.int64, device=pipe.m.device)
    ws = cga.Workspaces(pipe.m.device)
    run = lambda: cga.cga_occupancy(pipe.m, pipe.g, n=n, occ_out=occ, counts_out=counts, sync=False,
                                    ws=ws)
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    codes = int(counts[1:].sum().item())
    return {"keys": n, "codes": codes, "ms": round(ms, 4), "codes_per_s": codes / (ms * 1e-3)}


def _time_ms(run, reps):
    import torch
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def paper_array_ops(cga, pipe, d, reps=20):
    """The paper's own lookup and NN on the five arrays of the step's union in
    LINEAR order (not part of the step): the union rebuilt on a LINEAR grid,
    cga_to_arrays, then the three-level lookup of 2M voxels (half present)
    and the epsilon-box NN of the step's queries, next to the octree k-NN of
    the same queries with k = 1."""
    import numpy as np
    import torch

    import gen
    dev = pipe.m.device
    g = d["grid"].with_mode(gen.KEY_LINEAR)
    ka, _ = cga.cga_build(pipe.a, g)
    kb, _ = cga.cga_build(pipe.b, g)
    m, _ = cga.cga_merge(ka, kb, g)
    arr = cga.cga_to_arrays(m, g)
    n = m.shape[0]
    rng = np.random.default_rng(1008)
    mk = m.cpu().numpy().view(np.uint64)[rng.integers(0, n, 1 << 20)]
    dd = g.depth
    mask = (1 << dd) - 1
    present = np.stack([(mk >> np.uint64(2 * dd)) & np.uint64(mask), (mk >> np.uint64(dd)) & np.uint64(mask),
                        mk & np.uint64(mask)], 1)
    qv = np.concatenate([present, rng.integers(0, 1 << dd, (1 << 20, 3))]).astype(np.int32)
    qv = torch.from_numpy(qv).to(dev)
    pos = torch.empty(qv.shape[0], dtype=torch.int64, device=dev)
    nq = pipe.q.shape[0]
    idx = torch.empty(nq, dtype=torch.int64, device=dev)
    d2 = torch.empty(nq, dtype=torch.int64, device=dev)
    kidx = torch.empty((nq, 1), dtype=torch.int64, device=dev)
    kd2 = torch.empty((nq, 1), dtype=torch.int64, device=dev)
    ws = cga.Workspaces(dev)
    ms_lookup = _time_ms(lambda: cga.cga_arrays_lookup(arr, qv, g, out=pos, sync=False, ws=ws), reps)
    ms_nn = _time_ms(lambda: cga.cga_arrays_nn(arr, pipe.q, g, idx_out=idx, d2_out=d2, sync=False,
                                                ws=ws), reps)
    ms_knn1 = _time_ms(lambda: cga.cga_knn(pipe.m, pipe.q, pipe.g, 1, n=pipe.nu, idx_out=kidx,
                                           d2_out=kd2, sync=False, ws=ws), reps)
    torch.cuda.synchronize()
    same = bool(torch.equal(d2, kd2[:, 0]))
    return {"voxels": n, "x_entries": int(arr["x_index"].shape[0]),
            "xy_entries": int(arr["y_index"].shape[0]),
            "lookup": {"queries": int(qv.shape[0]), "ms": round(ms_lookup, 4),
                       "lookups_per_s": qv.shape[0] / (ms_lookup * 1e-3),
                       "found": int((pos >= 0).sum().item())},
            "nn": {"queries": nq, "ms": round(ms_nn, 4), "queries_per_s": nq / (ms_nn * 1e-3)},
            "octree_knn_k1": {"ms": round(ms_knn1, 4), "queries_per_s": nq / (ms_knn1 * 1e-3),
                              "same_distances": same}}


def temporal_prediction(cga, device, reps=5):
    """One inter-frame step of the CGA compression scheme (not part of the
    step): the moving-object frame pair (about 5.4e5 voxels per frame on a
    1024^3 grid), both frames built with their Value arrays, then k-means,
    motion vectors, SAD matching and residuals (window 2, at most 100
    passes), timed as one cga_temporal_predict call."""
    import numpy as np
    import torch

    import gen
    d = gen.c6_frames()
    g = d["grid"]

    def frame(xyz, cols):
        x = torch.from_numpy(xyz).to(device)
        keys, _ = cga.cga_build(x, g)
        vals = cga.cga_voxel_values(x, torch.from_numpy(cols.view(np.int32)).to(device), keys, g)
        return keys, vals

    rk, rv = frame(d["ref"], d["ref_values"])
    pk, pv = frame(d["pred"], d["pred_values"])
    out = cga.cga_temporal_predict(rk, rv, pk, pv, g, window=2, max_iter=100)
    ws = cga.Workspaces(device)
    ms = _time_ms(lambda: cga.cga_temporal_predict(rk, rv, pk, pv, g, window=2, max_iter=100,
                                                   out=out, sync=False, ws=ws), reps)
    torch.cuda.synchronize()
    res = out["residual"][:pk.shape[0], :3].abs().float().mean().item()
    matched = (out["match"][:pk.shape[0]] >= 0).float().mean().item()
    return {"ref_voxels": int(rk.shape[0]), "pred_voxels": int(pk.shape[0]),
            "passes": out["iters"].cpu().tolist(), "ms": round(ms, 3),
            "voxels_per_s": (rk.shape[0] + pk.shape[0]) / (ms * 1e-3),
            "matched": round(matched, 4), "mean_abs_rgb_residual": round(res, 3)}


def attribute_values(cga, pipe, d, reps=20):
    """Value arrays of the step's two sweeps from seeded per-point attributes,
    and the merged cloud's values (average policy); not part of the step."""
    import torch

    import gen
    dev = pipe.m.device
    aa = torch.from_numpy(gen.attributes(1007, 1, pipe.na).view("int32")).to(dev)
    ab = torch.from_numpy(gen.attributes(1007, 2, pipe.nb).view("int32")).to(dev)
    ua, ub, um = [int(x) for x in pipe.cnt[:3].cpu().tolist()]
    va = torch.empty(max(ua, 1), dtype=torch.int32, device=dev)
    vb = torch.empty(max(ub, 1), dtype=torch.int32, device=dev)
    vm = torch.empty(max(um, 1), dtype=torch.int32, device=dev)
    ws = cga.Workspaces(dev)

    def run():
        cga.cga_voxel_values(pipe.a, aa, pipe.ka, pipe.g, u=ua, out=va, sync=False, ws=ws)
        cga.cga_voxel_values(pipe.b, ab, pipe.kb, pipe.g, u=ub, out=vb, sync=False, ws=ws)
        cga.cga_merge_values(pipe.ka, va, pipe.kb, vb, pipe.m, pipe.g, cga.VALUES_AVERAGE, na=ua,
                             nb=ub, nm=um, out=vm, sync=False, ws=ws)
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"points": pipe.na + pipe.nb, "voxels": [ua, ub, um], "ms": round(ms, 4),
            "points_per_s": (pipe.na + pipe.nb) / (ms * 1e-3)}


def c4_batched(cga, device, reps):
    """256 LiDAR frames (log-uniform 10k..2M points) built and pair-merged by
    one replay of the captured graph; the sort's digit width and tile size
    come from the autotuner run on the same number of keys."""
    import numpy as np
    import torch

    import gen
    t0 = time.perf_counter()
    d = gen.c4_frames()
    xyz = torch.from_numpy(d["xyz"]).to(device)
    off = torch.from_numpy(d["off"]).to(device)
    g = d["grid"]
    n, F = len(xyz), len(off) - 1
    gen_s = time.perf_counter() - t0
    fb = int(np.ceil(np.log2(F)))
    rb, items, tune_ms = cga.cga_autotune_sort(key_bytes=8, key_bits=3 * g.depth + fb, n=n)
    graph = cga.BatchGraph(xyz, off, g)
    graph.launch()
    torch.cuda.synchronize()
    if graph.status() != 0:
        raise RuntimeError("batched graph reported an error")
    # the graph's frame 0 and pair 0 against the standalone entry points
    k0, _ = cga.cga_build(xyz[: int(d["off"][1])], g)
    k1, _ = cga.cga_build(xyz[int(d["off"][1]): int(d["off"][2])], g)
    m01, _ = cga.cga_merge(k0, k1, g)
    same = bool(torch.equal(graph.out.frame(0), k0) and torch.equal(graph.out.pair(0), m01))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        graph.launch()
        b.record()
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    u = int(graph.out.key_off[-1].item())
    merged = int(graph.out.merged_cnt[: F - 1].sum().item())
    graph.close()
    return {"frames": F, "points": n, "unique_total": u, "merged_total": merged,
            "gen_s": round(gen_s, 1), "autotune": {"radix_bits": rb, "tile_items": items,
                                                   "sort_ms": round(tune_ms, 3)},
            "graph_ms": round(ms, 3), "points_per_s": n / (ms * 1e-3),
            "frame0_pair0_match_standalone": same}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path is single-GPU; see the sharding design notes)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import torch

    import paper_2110_11616_amd as cga
    device = torch.device("cuda:0")
    d = make_workload(args.workload)
    pipe = Pipeline(cga, d, device)

    pipe.step()
    torch.cuda.synchronize()
    pipe.check()
    pipe.nu = int(pipe.cnt[2].item())
    pipe.make_lookups()
    for _ in range(args.warmup):
        pipe.step()
        pipe.step_concurrent()
    torch.cuda.synchronize()
    pipe.check()
    counts = [int(x) for x in pipe.cnt.cpu().tolist()]
    if not (torch.equal(pipe.lrank, pipe.brank) and torch.equal(pipe.lfound, pipe.bfound)):
        raise RuntimeError("learned and binary lookups disagree")

    # per-kernel breakdown (untimed pass), to name the dominant kernel
    labels = ["begin", "encode", "histogram", "hist_scan", "onesweep", "rle", "merge_partition",
              "merge", "rekey", "knn_tree", "knn", "index_root", "index_bounds", "index_fit", "index_err",
              "index_lookup", "binary_lookup"]
    kern_ms = {}
    dominant = None
    if not args.no_kernel_timing:
        cga.cga_prof_reset()
        cga.cga_prof_enable(None)
        for _ in range(2):
            pipe.step()
        torch.cuda.synchronize()
        cga.cga_prof_disable()
        for lb in labels:
            ms, n = cga.cga_prof_read(lb)
            if n:
                kern_ms[lb] = round(ms / 2, 4)
        cga.cga_prof_reset()
        dominant = max(kern_ms, key=kern_ms.get) if kern_ms else None
        if dominant:
            cga.cga_prof_enable([dominant])

    # the timed steps: independent parts overlapped on side streams
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for s in range(args.steps):
        pipe.step_concurrent()
    stop.record()
    torch.cuda.synchronize()
    cga.cga_prof_disable()
    pipe.check()
    if not (torch.equal(pipe.lrank, pipe.brank) and torch.equal(pipe.lfound, pipe.bfound)):
        raise RuntimeError("learned and binary lookups disagree")
    ms_eager = start.elapsed_time(stop) / args.steps
    ms_graph = graph_step(pipe, args.steps)
    ms = ms_graph

    # stage breakdown: the same steps one part after the other on one stream
    marks = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(args.steps)]
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s0.record()
    for s in range(args.steps):
        pipe.step(marks[s])
    s1.record()
    torch.cuda.synchronize()
    pipe.check()
    ms_serial = s0.elapsed_time(s1) / args.steps

    def stage(i, j):
        return sum(m[i].elapsed_time(m[j]) for m in marks) / args.steps

    st_build = stage(0, 1)
    st_proj = stage(1, 2)
    st_knn = stage(2, 3)
    st_train = stage(3, 4)
    st_learned = stage(4, 5)
    st_binary = stage(5, 6)
    n_points = pipe.na + pipe.nb
    nq = len(pipe.q)

    roofline = None
    if dominant:
        tot_ms, launches = cga.cga_prof_read(dominant)
        algo = algorithmic_bytes(dominant, pipe, counts)
        if algo is not None and launches:
            per_step_launches = launches / args.steps
            avg_ms = tot_ms / launches
            bytes_per_launch = algo / per_step_launches
            achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
            traffic = load_traffic(dominant, args.workload)
            roofline = {
                "bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic) if traffic else None,
                "avg_launch_us": round(avg_ms * 1e3, 2), "launches_per_step": per_step_launches,
                # events bracket the launches of the overlapped step issued
                # per step (they cannot sit inside the replayed graph, where
                # the search shares the GPU with the leaf training more tightly)
                "measured_on": "overlapped step, launched per step",
                "algorithmic_bytes_per_launch": round(bytes_per_launch),
            }
        cga.cga_prof_reset()
    # context for the other kernels of the step that move bytes: algorithmic
    # bytes per step over their measured time per step (untimed warm passes
    # above), next to the same HBM peak and, where counted, their traffic
    by_kernel = {}
    for lb, kms in kern_ms.items():
        algo = algorithmic_bytes(lb, pipe, counts)
        if algo is None or kms <= 0:
            continue
        gbs = algo / (kms * 1e-3) / 1e9
        by_kernel[lb] = {"ms_per_step": kms, "algorithmic_mb_per_step": round(algo / 1e6, 2),
                         "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}

    line = {
        "metric": "CGA build+merge points/s & kNN queries/s at % HBM peak; learned vs binary lookup/s",
        "value": n_points / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "ms_per_step_eager": round(ms_eager, 4), "ms_per_step_serial": round(ms_serial, 4),
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64" if 3 * pipe.g.depth > 32 else "u32",
        "data": "synthetic",
        "config": {"workload": {"c1": "c1_spheres_100k_d10", "c2": "c2_lidar_2x1048576_d12",
                                "c3": "c3_bumpy_2x10M_d14"}[args.workload],
                   "points_per_step": n_points, "queries": nq, "k": pipe.k,
                   "depth": pipe.g.depth, "unique": counts,
                   "streams": "build A | build B, merge, then projection | k-NN | index "
                              "training + lookups, captured once as one HIP graph and replayed "
                              "(eager: the same launches issued per step; stages: the same "
                              "step on one stream)"},
        "stages": {
            "build_merge": {"ms": round(st_build, 4), "points_per_s": n_points / (st_build * 1e-3)},
            "project_xy": {"ms": round(st_proj, 4)},
            "knn": {"ms": round(st_knn, 4), "queries_per_s": nq / (st_knn * 1e-3)},
            "index_train": {"ms": round(st_train, 4), "keys": pipe.nu},
            "learned_lookup": {"ms": round(st_learned, 4),
                               "lookups_per_s": pipe.nl / (st_learned * 1e-3)},
            "binary_lookup": {"ms": round(st_binary, 4),
                              "lookups_per_s": pipe.nl / (st_binary * 1e-3)},
        },
        "kernels_ms_per_step": kern_ms,
        "roofline": roofline,
        "hbm_by_kernel": by_kernel,
        "cpu_baseline": None,
    }
    line["occupancy"] = occupancy_codes(cga, pipe)
    line["values"] = attribute_values(cga, pipe, d)
    line["paper_array_ops"] = paper_array_ops(cga, pipe, d)
    line["temporal"] = temporal_prediction(cga, device)
    if not args.no_c5:
        line["c5"] = c5_learned_vs_binary(cga, device, args.c5_reps)
    if not args.no_c4:
        line["c4"] = c4_batched(cga, device, args.c4_reps)
    if not args.no_cpu_baseline:
        import numpy as np
        line["cpu_baseline"] = cpu_baseline(d, pipe.lq.cpu().numpy().view(np.uint64))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
