#!/usr/bin/env python3
"""Benchmark of the CGA hot path on one MI355X.

One step = the whole pipeline on one batch of synthetic input, already in
HBM: build the CGA of two LiDAR sweeps (quantize, encode, radix sort,
run-length compaction), merge them, project the union onto XY, and answer
k-NN queries against the union.  Workloads:
  c2 (default): 2 x 1,048,576-point sweeps, depth 12, 100k queries, k = 8
  c3: 2 x 10M-point bumpy spheres, depth 14, 1M queries, k = 16
  c1: 2 x 100k sphere points, depth 10, 1k queries, k = 1
Prints one JSON line.  value = input points per second of whole steps.
"""
from __future__ import annotations

import argparse
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
    return ap.parse_args()


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
        self.ws = [cga.Workspaces(device) for _ in range(5)]

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

    def check(self):
        for w in self.ws:
            for buf in w.bufs.values():
                st = self.cga.lib.cga_ws_status(self.cga._ptr(buf), self.cga._stream())
                if st != 0:
                    raise self.cga.CgaError(st, "bench step")


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
    """HBM bytes per step of a kernel from committed rocprofv3 counter runs,
    or None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{label}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_step")


def cpu_baseline(d):
    """The oracle, untuned, on one full step of the same workload."""
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
                   f"k-NN on {threads} OpenMP threads ({t_knn / steps:.2f} s/step)"),
        "seconds_per_step": round(per, 3),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path is single-GPU; see the sharding design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2110_11616_amd as cga
    device = torch.device("cuda:0")
    d = make_workload(args.workload)
    pipe = Pipeline(cga, d, device)

    for _ in range(args.warmup):
        pipe.step()
    torch.cuda.synchronize()
    pipe.check()
    counts = [int(x) for x in pipe.cnt.cpu().tolist()]

    # per-kernel breakdown (untimed pass), to name the dominant kernel
    labels = ["begin", "encode", "histogram", "hist_scan", "onesweep", "rle", "merge_partition",
              "merge", "rekey", "knn"]
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

    marks = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for s in range(args.steps):
        pipe.step(marks[s])
    stop.record()
    torch.cuda.synchronize()
    cga.cga_prof_disable()
    pipe.check()
    ms = start.elapsed_time(stop) / args.steps

    def stage(i, j):
        return sum(m[i].elapsed_time(m[j]) for m in marks) / args.steps

    st_build = stage(0, 1)
    st_proj = stage(1, 2)
    st_knn = stage(2, 3)
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
                "traffic": (round(traffic / per_step_launches) if traffic else None),
                "avg_launch_us": round(avg_ms * 1e3, 2), "launches_per_step": per_step_launches,
                "algorithmic_bytes_per_launch": round(bytes_per_launch),
            }
        cga.cga_prof_reset()

    line = {
        "metric": "CGA build+merge points/s & kNN queries/s at % HBM peak; learned vs binary lookup/s",
        "value": n_points / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64" if 3 * pipe.g.depth > 32 else "u32",
        "data": "synthetic",
        "config": {"workload": {"c1": "c1_spheres_100k_d10", "c2": "c2_lidar_2x1048576_d12",
                                "c3": "c3_bumpy_2x10M_d14"}[args.workload],
                   "points_per_step": n_points, "queries": nq, "k": pipe.k,
                   "depth": pipe.g.depth, "unique": counts},
        "stages": {
            "build_merge": {"ms": round(st_build, 4), "points_per_s": n_points / (st_build * 1e-3)},
            "project_xy": {"ms": round(st_proj, 4)},
            "knn": {"ms": round(st_knn, 4), "queries_per_s": nq / (st_knn * 1e-3)},
        },
        "kernels_ms_per_step": kern_ms,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(d)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
