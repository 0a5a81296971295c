#!/usr/bin/env python3
"""Benchmark of the CGA hot path on one MI355X.

One step = the whole pipeline on one batch of synthetic input, already in
HBM: build the CGA of two clouds (quantize, encode, radix sort, run-length
compaction), merge them, project the union onto the axis planes, answer k-NN
queries against the union, train the learned index of the union and answer
point-location / range-start lookups with it and with binary search.
Workloads:
  c3 (default): 2 x 10M bumpy-sphere points, depth 14, projections along all
      three axes, 1M queries, k = 16
  c2: 2 x 1,048,576-point LiDAR sweeps, depth 12, XY projection, 100k
      queries, k = 8
  c1: 2 x 100k sphere points, depth 10, XY projection, 1k queries, k = 1
Prints one JSON line.  value = build+merge points per second: input points
of both clouds over the time of the build of both clouds and their merge,
measured over `steps` graph replays of exactly that part (the roofline
object is its dominant kernel, the radix sort pass).  ms_per_step is the
whole step (every part above, overlapped, one graph replay per step); the
k-NN queries per second and their two rooflines are reported under "knn".
Unless --no-c5, it also measures the learned index against binary search on
the 50M-key, 10M-query configuration ("c5"); unless --no-c4 the graph-captured
batched build + pair merge of 256 LiDAR frames ("c4", with its own roofline);
unless --no-legs the Value array, occupancy codes, the paper's array
operations and the temporal-prediction step on the c2 LiDAR union and the c6
frame pair ("legs"); and the attainable copy bandwidth of the GPU
("stream_probe").  None of these enter value.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Wave64 VALU instructions per second: 256 CUs x 4 SIMDs x 2.4 GHz, one
# wave64 instruction per SIMD every 4 cycles (16 lanes wide).
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4
T0 = time.perf_counter()

WORKLOADS = {
    # name: (workload label, projection axes dropped)
    "c1": ("c1_spheres_100k_d10", (2,)),
    "c2": ("c2_lidar_2x1048576_d12", (2,)),
    "c3": ("c3_bumpy_2x10M_d14", (0, 1, 2)),
}


def progress(msg):
    """One progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.perf_counter() - T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the per-kernel event timing (for external profilers)")
    ap.add_argument("--no-c5", action="store_true", help="skip the 50M-key learned-index run")
    ap.add_argument("--c5-reps", type=int, default=10)
    ap.add_argument("--no-c4", action="store_true", help="skip the 256-frame batched run")
    ap.add_argument("--c4-reps", type=int, default=5)
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the Value / occupancy / paper-array / temporal legs")
    ap.add_argument("--no-probe", action="store_true", help="skip the bandwidth probe")
    ap.add_argument("--autotune", action="store_true",
                    help="run the sort autotuner on this workload's key sizes first")
    ap.add_argument("--sort-tune", default="", metavar="RB,ITEMS,RB2,ITEMS2",
                    help="use these sort settings for the builds (RB, ITEMS) and projections "
                         "(RB2, ITEMS2) instead of running the autotuner (profiling runs)")
    ap.add_argument("--only", default="", choices=["", "build_merge", "step", "knn", "c4"],
                    help="time only this part (for external profilers)")
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
    return {"c1": gen.c1_spheres, "c2": gen.c2_lidar, "c3": gen.c3_bumpy}[name]()


class Pipeline:
    """Preallocated buffers and workspaces for one step; every size stays on
    the device between calls.  cnt = [U_a, U_b, U_union, pixels per
    projection...]."""

    def __init__(self, cga, d, device, drops=(2,)):
        import torch
        self.cga, self.g, self.k = cga, d["grid"], d["k"]
        self.drops = tuple(drops)
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
        self.p = [e(self.nm, k2t) for _ in self.drops]
        self.pc = [e(self.nm, torch.int32) for _ in self.drops]
        nq = len(self.q)
        self.idx = torch.empty((nq, self.k), dtype=torch.int64, device=device)
        self.d2 = torch.empty((nq, self.k), dtype=torch.int64, device=device)
        self.cnt = torch.zeros(3 + len(self.drops), dtype=torch.int64, device=device)
        # workspaces: build A, build B, merge, knn, index train, index lookup,
        # then one per projection
        self.ws = [cga.Workspaces(device) for _ in range(6 + len(self.drops))]
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
        self.nu = None
        self.lrank = torch.empty(self.nl, dtype=torch.int64, device=device)
        self.lfound = torch.empty(self.nl, dtype=torch.uint8, device=device)
        self.brank = torch.empty(self.nl, dtype=torch.int64, device=device)
        self.bfound = torch.empty(self.nl, dtype=torch.uint8, device=device)
        self.fb = torch.zeros(1, dtype=torch.int64, device=device)
        # side streams (default priority) for the independent parts of a step
        self.side = [torch.cuda.Stream(device=device) for _ in range(3 + len(self.drops))]
        self.tune_build = self.tune_proj = None  # (radix bits, tile items) or None
        self.ev = [torch.cuda.Event() for _ in range(6 + len(self.drops))]

    def make_lookups(self, seed=1006):
        import numpy as np
        import torch

        import gen
        self.nu = int(self.cnt[2].item())
        m = self.m[: self.nu].cpu().numpy().view(np.uint64)
        self.lq = torch.from_numpy(gen.lookup_queries(seed, m, self.nl).view(np.int64)).to(
            self.m.device)

    # -- parts of a step (each enqueued on the current stream)
    def _build(self, which):
        c, g, cnt = self.cga, self.g, self.cnt
        if which == 0:
            c.cga_build(self.a, g, keys_out=self.ka, counts_out=self.ca, d_n_out=cnt[0:1],
                        sync=False, ws=self.ws[0], tune=self.tune_build)
        else:
            c.cga_build(self.b, g, keys_out=self.kb, counts_out=self.cb, d_n_out=cnt[1:2],
                        sync=False, ws=self.ws[1], tune=self.tune_build)

    def _merge(self):
        c, cnt = self.cga, self.cnt
        c.cga_merge(self.ka, self.kb, self.g, na=self.na, d_na=cnt[0:1], nb=self.nb, d_nb=cnt[1:2],
                    out=self.m, d_n_out=cnt[2:3], sync=False, ws=self.ws[2])

    def _project(self, i):
        c, cnt = self.cga, self.cnt
        c.cga_project(self.m, self.g, self.drops[i], n=self.nm, d_n=cnt[2:3], out=self.p[i],
                      counts_out=self.pc[i], d_n_out=cnt[3 + i:4 + i], sync=False,
                      ws=self.ws[6 + i], tune=self.tune_proj)

    def _knn(self):
        self.cga.cga_knn(self.m, self.q, self.g, self.k, n=self.nm, d_n=self.cnt[2:3],
                         idx_out=self.idx, d2_out=self.d2, sync=False, ws=self.ws[3])

    def _index_train(self):
        # the index is trained on the union; its size comes from the host
        # copy taken at setup (the merge result is identical every step)
        self.cga.cga_index_train(self.m, self.nu, out=self.index, ws=self.ws[4],
                                 **self.index_kwargs)

    def _lookups(self, marks=None, i=0):
        c = self.cga
        c.cga_index_lookup(self.index, self.m, self.lq, n=self.nu, rank_out=self.lrank,
                           found_out=self.lfound, fallbacks_out=self.fb, sync=False, ws=self.ws[5])
        if marks:
            marks[i].record()
        c.cga_binary_lookup(self.m, self.lq, n=self.nu, rank_out=self.brank, found_out=self.bfound)

    def build_merge(self):
        """Build both clouds and merge them, one part after the other."""
        self._build(0)
        self._build(1)
        self._merge()

    def build_merge_concurrent(self):
        """The two builds side by side (second on a side stream), then the merge."""
        import torch
        main = torch.cuda.current_stream()
        sb = self.side[0]
        self.ev[0].record(main)
        sb.wait_event(self.ev[0])
        self._build(0)
        with torch.cuda.stream(sb):
            self._build(1)
        self.ev[1].record(sb)
        main.wait_event(self.ev[1])
        self._merge()

    def step(self, marks=None):
        """The whole step on one stream; marks (events) split it into
        build+merge | projections | k-NN | index training | learned lookups |
        binary lookups."""
        if marks:
            marks[0].record()
        self.build_merge()
        if marks:
            marks[1].record()
        for i in range(len(self.drops)):
            self._project(i)
        if marks:
            marks[2].record()
        self._knn()
        if marks:
            marks[3].record()
        if self.lq is not None:
            self._index_train()
            if marks:
                marks[4].record()
            self._lookups(marks, 5)
            if marks:
                marks[6].record()

    def step_concurrent(self):
        """The same step with its independent parts overlapped on side
        streams: the two builds side by side, then the merge, then the
        projections, the k-NN search and the index training + lookups side
        by side; the step ends when all have (the next step's builds
        overwrite what they read)."""
        import torch
        main = torch.cuda.current_stream()
        self.build_merge_concurrent()
        ev = self.ev
        ev[2].record(main)
        sk, si = self.side[1], self.side[2]
        sps = self.side[3:]
        for s in (sk, si, *sps):
            s.wait_event(ev[2])
        # the k-NN search, the longest branch, is issued first
        with torch.cuda.stream(sk):
            self._knn()
        for i, sp in enumerate(sps):
            with torch.cuda.stream(sp):
                self._project(i)
        with torch.cuda.stream(si):
            self._index_train()
            self._lookups()
        for e, s in zip(ev[3:], (sk, si, *sps)):
            e.record(s)
            main.wait_event(e)

    def check(self):
        for w in self.ws:
            for buf in w.bufs.values():
                st = self.cga.lib.cga_ws_status(self.cga._ptr(buf), self.cga._stream())
                if st != 0:
                    raise self.cga.CgaError(st, "bench step")


def step_outputs(pipe, full=True):
    """Copies of everything one step (or its build+merge part) writes, the
    arrays up to their counts."""
    cnt = pipe.cnt.tolist()
    ua, ub, um = cnt[:3]
    out = [pipe.cnt[:3].clone(), pipe.ka[:ua].clone(), pipe.ca[:ua].clone(), pipe.kb[:ub].clone(),
           pipe.cb[:ub].clone(), pipe.m[:um].clone()]
    if full:
        out.append(pipe.cnt.clone())
        for i in range(len(pipe.drops)):
            up = cnt[3 + i]
            out += [pipe.p[i][:up].clone(), pipe.pc[i][:up].clone()]
        out += [t.clone() for t in (pipe.idx, pipe.d2, pipe.index, pipe.lrank, pipe.lfound,
                                    pipe.brank, pipe.bfound)]
    return out


def graph_replay(pipe, fn, steps, full):
    """fn captured once into a HIP graph (side streams become branches) and
    replayed: the same kernels, launched without per-kernel host work.  Every
    output of the first replay and of the last timed one must equal an eager
    run's, with eager runs and synchronisations in between.  Returns ms per
    replay."""
    import torch
    fn()
    torch.cuda.synchronize()
    want = step_outputs(pipe, full)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(graph, stream=cap):
        fn()
    torch.cuda.synchronize()

    def same():
        got = step_outputs(pipe, full)
        return all(torch.equal(a, b) for a, b in zip(got, want))

    graph.replay()
    torch.cuda.synchronize()
    if not same():
        raise RuntimeError("graph replay differs from the eager run")
    fn()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        graph.replay()
    stop.record()
    torch.cuda.synchronize()
    pipe.check()
    if not same():
        raise RuntimeError("graph replay differs from the eager run")
    del graph
    return start.elapsed_time(stop) / steps


def sort_passes(bits, rb=8):
    return -(-bits // rb)


def library_sort_default(key_bytes, key_bits, n):
    """The library's default (radix bits, tile items) for a sort (restated
    here for the report): the fewest passes 8-bit digits allow, each as
    narrow as that count permits; 16 items per thread below 2^22 keys, else
    24 (64-bit keys) or 32 (32-bit keys)."""
    passes = sort_passes(key_bits)
    rb = max(4, -(-key_bits // passes))
    items = 16 if n < (1 << 22) else (24 if key_bytes == 8 else 32)
    return rb, items


def algorithmic_bytes(label, pipe, counts, build_merge_only=False, rb=(8, 8)):
    """Bytes the method itself must move for a kernel label over one step
    (reads + writes of its essential inputs and outputs); build_merge_only
    restricts it to the build + merge part; rb = the digit widths of the
    build's and the projections' sorts."""
    kb = 8 if 3 * pipe.g.depth > 32 else 4
    k2b = 8 if 2 * pipe.g.depth > 32 else 4
    passes3 = sort_passes(3 * pipe.g.depth, rb[0])
    passes2 = sort_passes(2 * pipe.g.depth, rb[1])
    ua, ub, um = counts[:3]
    ups = counts[3:] if not build_merge_only else []
    nproj = len(ups)
    if label == "onesweep":
        # every pass reads and writes each key once
        return passes3 * 2 * kb * (pipe.na + pipe.nb) + nproj * passes2 * 2 * k2b * um
    if label == "encode":
        return (12 + kb) * (pipe.na + pipe.nb)
    if label == "rle":
        return (kb * (pipe.na + pipe.nb) + (kb + 4) * (ua + ub)
                + sum(k2b * um + (k2b + 4) * up for up in ups))
    if label == "merge":
        return kb * (ua + ub + um)
    if build_merge_only:
        return None
    if label == "rekey":
        return nproj * (kb + k2b) * um
    if label == "knn_tree":
        # read every key of the union once
        return kb * um
    if label == "knn":
        # lower bound without the search's own reads: each query read (12 B)
        # and its k (index, d2) pairs written (16 B each); the full figure,
        # with the node words the search loads, comes from the counting build
        return len(pipe.q) * (12 + 16 * pipe.k)
    return None


def kernel_source_sha():
    import glob
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2110_11616_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def load_profile_json(label, workload, kind="traffic"):
    """A committed rocprofv3 counter summary (profiles/<label>_<workload>_<kind>.json),
    or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{label}_{workload}_{kind}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t


def load_traffic(label, workload):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a plain
    copy of known size), or None when absent or taken on other kernel sources."""
    t = load_profile_json(label, workload)
    return t.get("bytes_per_launch") if t else None


def cpu_info():
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def cpu_baseline(d, workload, lookups=None):
    """The oracle, untuned, on a bounded sample of the same workload (the
    learned index has no oracle counterpart beyond lower_bound itself)."""
    import numpy as np

    import oracle
    g = d["grid"]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    info = cpu_info()
    if workload != "c3":
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
        per = (t_set + t_knn) / steps
        return {
            "value": n / per, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": (f"{steps} full step(s) of {n} points and {len(d['q'])} queries: "
                       f"std::map/std::set build, merge and projection on 1 thread "
                       f"({t_set / steps:.2f} s/step), kd-tree k-NN and lower_bound lookups on "
                       f"{threads} OpenMP threads ({t_knn / steps:.2f} s/step)"),
            "seconds_per_step": round(per, 3), **info,
        }
    # c3: the full step would take minutes of CPU time; time the oracle's
    # build + merge on the first 1M points of each cloud (1 thread, std::map
    # and std::set_union) and its kd-tree k-NN of 20k seeded queries over the
    # whole union (tree build included, OpenMP over the queries)
    ns = 1_000_000
    t0 = time.perf_counter()
    ka, _ = oracle.build(d["a"][:ns], g)
    kb, _ = oracle.build(d["b"][:ns], g)
    oracle.merge(ka, kb, g.depth, g.key_mode)
    t_bm = time.perf_counter() - t0
    union = np.union1d(np.unique(oracle.encode(oracle.quantize(d["a"], g), g.depth, g.key_mode)),
                       np.unique(oracle.encode(oracle.quantize(d["b"], g), g.depth, g.key_mode)))
    rows = np.sort(np.random.default_rng(3003).choice(len(d["q"]), 20_000, replace=False))
    t0 = time.perf_counter()
    oracle.knn_kdtree(union, d["q"][rows], g, d["k"])
    t_knn = time.perf_counter() - t0
    return {
        "value": 2 * ns / t_bm, "unit": "points/s", "cores": threads, "kind": "oracle",
        "sample": (f"build (std::map) of the first {ns} points of each cloud and their merge "
                   f"(std::set_union), 1 thread: {t_bm:.2f} s; kd-tree k-NN (k = {d['k']}) of "
                   f"{len(rows)} seeded queries over the whole {len(union)}-voxel union, tree "
                   f"build included, {threads} OpenMP threads: {t_knn:.2f} s"),
        "knn_queries_per_s": len(rows) / t_knn,
        "seconds": round(t_bm + t_knn, 2), **info,
    }


def stream_probe(cga, device, nbytes=2 << 30, reps=5):
    """Attainable HBM bandwidth: the library's plain copy and read kernels
    over 2 GiB buffers (far beyond the 256 MB Infinity Cache), best over
    launch widths."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device=device)
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.int32, device=device)
    best = {"copy": (0.0, 0), "read": (0.0, 0)}
    for blocks in (1024, 2048, 4096, 8192, 16384):
        for mode, name, moved in ((0, "copy", 2 * nbytes), (1, "read", nbytes)):
            other = dst if mode == 0 else sink
            cga.cga_stream_probe(src, other, nbytes, mode, blocks)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                cga.cga_stream_probe(src, other, nbytes, mode, blocks)
            e1.record()
            torch.cuda.synchronize()
            gbs = moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
            if gbs > best[name][0]:
                best[name] = (gbs, blocks)
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_gbs": round(best["copy"][0], 1), "copy_blocks": best["copy"][1],
            "read_gbs": round(best["read"][0], 1), "read_blocks": best["read"][1],
            "bytes": nbytes, "datasheet_gbs": HBM_PEAK_GBS,
            "copy_frac_of_datasheet": round(best["copy"][0] / HBM_PEAK_GBS, 3)}


def roofline_from_prof(label, algo_bytes, steps, traffic=None, note=""):
    """HBM roofline of one kernel label from the live HIP-event timing: its
    algorithmic bytes per launch over its average launch duration."""
    import paper_2110_11616_amd as cga
    tot_ms, launches = cga.cga_prof_read(label)
    if not launches or algo_bytes is None:
        return None
    per_step_launches = launches / steps
    avg_ms = tot_ms / launches
    bytes_per_launch = algo_bytes / per_step_launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return {
        "bound": "hbm", "kernel": label, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": round(traffic) if traffic else None,
        "avg_launch_us": round(avg_ms * 1e3, 2), "launches_per_step": per_step_launches,
        "algorithmic_bytes_per_launch": round(bytes_per_launch), "measured_on": note,
    }


def knn_work(cga, pipe):
    """The counting build of the search on the step's union and queries:
    identical results, plus the exact work per query."""
    import torch
    idx, d2, w = cga.cga_knn_count(pipe.m, pipe.q, pipe.g, pipe.k, n=pipe.nm, d_n=pipe.cnt[2:3])
    torch.cuda.synchronize()
    if not (torch.equal(idx, pipe.idx) and torch.equal(d2, pipe.d2)):
        raise RuntimeError("the counting k-NN build disagrees with the search")
    nq = len(pipe.q)
    return {k: v / nq for k, v in w.items()}


def c2_context(cga, device, steps):
    """The LiDAR sweep pair (c2) at its own size: build+merge points/s and
    k-NN queries/s, for context beside the headline workload."""
    import torch
    d = make_workload("c2")
    pipe = Pipeline(cga, d, device, WORKLOADS["c2"][1])
    pipe.step()
    torch.cuda.synchronize()
    pipe.check()
    ms_bm = graph_replay(pipe, pipe.build_merge_concurrent, steps, False)
    ms_knn = _time_ms(pipe._knn, steps)
    n = pipe.na + pipe.nb
    return pipe, d, {"workload": WORKLOADS["c2"][0], "build_merge_ms": round(ms_bm, 4),
                     "build_merge_points_per_s": n / (ms_bm * 1e-3),
                     "knn_ms": round(ms_knn, 4),
                     "knn_queries_per_s": len(pipe.q) / (ms_knn * 1e-3)}


C5_VARIANTS = (("linear_leaves_4096_root_linear", 0, 4096, 0),
               ("mlp_leaves_4096_root_linear", 1, 4096, 0),
               ("mlp_leaves_4096_pl1024", 1, 4096, 1024),
               ("linear_leaves_65536_pl4096", 0, 65536, 4096),
               ("mlp_leaves_65536_pl4096", 1, 65536, 4096),
               ("linear_leaves_1048576_pl4096", 0, 1 << 20, 4096),
               ("linear_leaves_4194304_pl4096", 0, 1 << 22, 4096),
               ("linear_leaves_16777216_pl4096", 0, 1 << 24, 4096))
C5_CONFIGURED = ("linear_leaves_4096_root_linear", "mlp_leaves_4096_root_linear")


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
                     "index_bytes": int(idx.numel()),
                     "index_bytes_per_key": round(idx.numel() / n, 3),
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
    ms_b = med(times["binary"])
    for name in res:
        fb.zero_()
        r, f, nfb = cga.cga_index_lookup(res[name]["idx"], keys, q, rank_out=rank_l,
                                        found_out=found_l, fallbacks_out=fb)
        cga.cga_binary_lookup(keys, q, rank_out=rank_b, found_out=found_b)
        torch.cuda.synchronize()
        same = bool(torch.equal(rank_l, rank_b) and torch.equal(found_l, found_b))
        if not same:
            raise RuntimeError(f"learned lookup ({name}) disagrees with binary search")
        ms = med(times[name])
        del res[name]["idx"]
        res[name].update({"lookup_ms": round(ms, 3), "lookups_per_s": len(q) / (ms * 1e-3),
                          "vs_binary": round(ms_b / ms, 3),
                          "fallback_rate": nfb / len(q), "identical_to_binary": same})
    out["binary"] = {"lookup_ms": round(ms_b, 3), "lookups_per_s": len(q) / (ms_b * 1e-3)}
    out["learned"] = res
    best = max(res, key=lambda k: res[k]["lookups_per_s"])
    out["best_learned"] = {"variant": best, "vs_binary": res[best]["vs_binary"],
                           "index_bytes_per_key": res[best]["index_bytes_per_key"]}
    out["configured_4096_leaves"] = {k: res[k]["vs_binary"] for k in C5_CONFIGURED if k in res}
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
    ms = _time_ms(run, reps)
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
    come from the autotuner run on the same number of keys.  Roofline: the
    method's bytes for every frame's build (quantize + encode, the autotuned
    number of sort passes over the key bits the frame-segmented sort covers,
    run-length compaction)
    and every pair's merge, over the replay time."""
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
    key_bits = cga.cga_batch_sort_bits(g, F)  # the bits the (frame-segmented) sort passes cover
    rb, items, tune_ms = cga.cga_autotune_sort(key_bytes=8, key_bits=key_bits, n=n)
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
    # per-kernel times of the same work launched eagerly (HIP events around
    # each launch; the graph itself cannot carry them)
    labels = ["batch_encode", "hist_scan", "onesweep", "rle", "batch_offsets", "batch_pairs",
              "batch_merge"]
    cga.cga_prof_reset()
    cga.cga_prof_enable(labels)
    for _ in range(2):
        cga.cga_batch_build_merge(xyz, off, g, tune=(rb, items))
    torch.cuda.synchronize()
    cga.cga_prof_disable()
    kern = {}
    for lb in labels:
        kms, kn = cga.cga_prof_read(lb)
        if kn:
            kern[lb] = {"ms_per_run": round(kms / 2, 4), "launches_per_run": kn // 2}
    if "onesweep" in kern and kern["onesweep"]["launches_per_run"]:
        us = kern["onesweep"]["ms_per_run"] * 1e3 / kern["onesweep"]["launches_per_run"]
        kern["onesweep"]["avg_launch_us"] = round(us, 1)
        kern["onesweep"]["gbs_per_pass"] = round(16 * n / (us * 1e-6) / 1e9, 1)
        kern["onesweep"]["algorithmic_bytes_per_pass"] = 16 * n
        kern["onesweep"]["traffic"] = load_traffic("onesweep", "c4")
    key_off = graph.out.key_off.cpu().numpy()
    uf = np.diff(key_off)
    u = int(key_off[-1])
    mc = graph.out.merged_cnt[: F - 1].cpu().numpy()
    merged = int(mc.sum())
    graph.close()
    S, P = 8, sort_passes(key_bits, rb)
    build_bytes = n * (12 + S + 2 * S * P + S) + u * (S + 4)
    merge_bytes = S * int((uf[:-1] + uf[1:]).sum() + merged)
    total = build_bytes + merge_bytes
    gbs = total / (ms * 1e-3) / 1e9
    return {"frames": F, "points": n, "unique_total": u, "merged_total": merged,
            "gen_s": round(gen_s, 1), "autotune": {"radix_bits": rb, "tile_items": items,
                                                   "sort_passes": P, "sort_ms": round(tune_ms, 3)},
            "graph_ms": round(ms, 3), "points_per_s": n / (ms * 1e-3), "kernels_eager": kern,
            "roofline": {"bound": "hbm", "kernel": "whole graph", "achieved": round(gbs, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes": total, "build_bytes": build_bytes,
                         "merge_bytes": merge_bytes},
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
    if args.only == "c4":
        # the 256-frame batched graph alone, replayed `steps` times
        c4 = c4_batched(cga, device, args.steps)
        progress(f"c4 only: graph {c4['graph_ms']} ms, onesweep {c4['kernels_eager'].get('onesweep')}")
        return
    wl_label, drops = WORKLOADS[args.workload]
    progress(f"generating workload {args.workload}")
    d = make_workload(args.workload)
    pipe = Pipeline(cga, d, device, drops)
    progress("inputs on the device")

    # the autotuner picks the sort's digit width and tile size for this
    # workload's key sizes (the cloud's own keys, and synthetic pixel keys
    # of the projections' width); builds and projections then use them
    kb2 = 8 if 2 * pipe.g.depth > 32 else 4
    if args.sort_tune:
        t = [int(x) for x in args.sort_tune.split(",")]
        tuned = {"build": (t[0], t[1], float("nan")), "project": (t[2], t[3], float("nan"))}
        pipe.tune_build, pipe.tune_proj = (t[0], t[1]), (t[2], t[3])
    elif args.autotune:
        tuned = {"build": cga.cga_autotune_sort(cga.cga_encode_keys(pipe.a, pipe.g),
                                                key_bits=3 * pipe.g.depth),
                 "project": cga.cga_autotune_sort(None, key_bytes=kb2, key_bits=2 * pipe.g.depth,
                                                  n=pipe.nm)}
    else:
        kb3 = 8 if 3 * pipe.g.depth > 32 else 4
        tuned = {"build": library_sort_default(kb3, 3 * pipe.g.depth, pipe.na) + (float("nan"),),
                 "project": library_sort_default(kb2, 2 * pipe.g.depth, pipe.nm) + (float("nan"),)}
    progress(f"sort settings (radix bits, tile items, tuned ms): {tuned}")
    pipe.step()
    torch.cuda.synchronize()
    pipe.check()
    pipe.make_lookups()
    for _ in range(args.warmup):
        pipe.step()
        pipe.step_concurrent()
    torch.cuda.synchronize()
    pipe.check()
    counts = [int(x) for x in pipe.cnt.cpu().tolist()]
    if not (torch.equal(pipe.lrank, pipe.brank) and torch.equal(pipe.lfound, pipe.bfound)):
        raise RuntimeError("learned and binary lookups disagree")
    progress(f"warm-up done; counts {counts}")

    if args.only:
        # one part only, launched `steps` times (profiler runs); the live
        # event timing of its main kernel is printed for comparison
        part = {"build_merge": (pipe.build_merge_concurrent, "onesweep"),
                "step": (pipe.step_concurrent, "knn"), "knn": (pipe._knn, "knn")}[args.only]
        if not args.no_kernel_timing:
            cga.cga_prof_reset()
            cga.cga_prof_enable([part[1]])
        for _ in range(args.steps):
            part[0]()
        torch.cuda.synchronize()
        cga.cga_prof_disable()
        ms, n = cga.cga_prof_read(part[1]) if not args.no_kernel_timing else (0.0, 0)
        progress(f"{args.only} only: done; {part[1]}: {n} launches, "
                 f"{ms / max(n, 1) * 1e3:.1f} us average (HIP events)")
        return

    # per-kernel breakdown (untimed serial steps)
    labels = ["begin", "encode", "histogram", "hist_scan", "onesweep", "rle", "merge_partition",
              "merge", "rekey", "knn_order", "knn_tree", "knn", "index_root", "index_bounds",
              "index_fit", "index_err", "index_lookup", "binary_lookup"]
    kern_ms = {}
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
        progress(f"per-kernel timing: {kern_ms}")

    rbs = (tuned["build"][0], tuned["project"][0])
    # build + merge: eager runs with the sort passes timed live (roofline),
    # then graph replays (value)
    n_points = pipe.na + pipe.nb
    bm_roof = None
    if not args.no_kernel_timing:
        cga.cga_prof_enable(["onesweep"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        pipe.build_merge_concurrent()
    e1.record()
    torch.cuda.synchronize()
    cga.cga_prof_disable()
    pipe.check()
    ms_bm_eager = e0.elapsed_time(e1) / args.steps
    if not args.no_kernel_timing:
        bm_roof = roofline_from_prof("onesweep", algorithmic_bytes("onesweep", pipe, counts, True,
                                                                   rbs),
                                     args.steps, load_traffic("onesweep", args.workload),
                                     "build+merge launched per run (both clouds' sort passes)")
        cga.cga_prof_reset()
    ms_bm = graph_replay(pipe, pipe.build_merge_concurrent, args.steps, False)
    progress(f"build+merge: eager {ms_bm_eager:.3f} ms, graph {ms_bm:.3f} ms")

    # the whole step: eager overlapped (k-NN search timed live), graph replay
    if not args.no_kernel_timing:
        cga.cga_prof_enable(["knn"])
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        pipe.step_concurrent()
    stop.record()
    torch.cuda.synchronize()
    cga.cga_prof_disable()
    pipe.check()
    if not (torch.equal(pipe.lrank, pipe.brank) and torch.equal(pipe.lfound, pipe.bfound)):
        raise RuntimeError("learned and binary lookups disagree")
    ms_eager = start.elapsed_time(stop) / args.steps
    progress(f"eager overlapped steps: {ms_eager:.3f} ms")
    knn_prof = cga.cga_prof_read("knn") if not args.no_kernel_timing else (0.0, 0)
    cga.cga_prof_reset()
    ms_graph = graph_replay(pipe, pipe.step_concurrent, args.steps, True)
    progress(f"graph-replayed steps: {ms_graph:.3f} ms")

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
    progress(f"serial steps: {ms_serial:.3f} ms")

    def stage(i, j):
        return sum(m[i].elapsed_time(m[j]) for m in marks) / args.steps

    st = [stage(i, i + 1) for i in range(6)]
    nq = len(pipe.q)

    # k-NN: the exact work per query (counting build), the HBM roofline with
    # those node loads, and the instruction-issue roofline from the committed
    # counter run of the same kernel sources
    work = knn_work(cga, pipe)
    progress(f"k-NN work per query: {work}")
    # a node visit reads the node's two words (mask and first child; oriented box)
    knn_bytes_q = 12 + 16 * pipe.k + 16 * work["node_loads"] + 4 * work["dense_loads"]
    knn = {"queries": nq, "k": pipe.k, "stage_ms": round(st[2], 4),
           "queries_per_s": nq / (st[2] * 1e-3),
           "work_per_query": {k: round(v, 2) for k, v in work.items()},
           "bytes_per_query": {"algorithmic": round(knn_bytes_q, 1),
                               "every_node_load_a_line": round(12 + 16 * pipe.k + 128 * (
                                   work["node_loads"] + work["dense_loads"]), 1)}}
    if knn_prof[1]:
        avg_ms = knn_prof[0] / knn_prof[1]
        achieved = nq * knn_bytes_q / (avg_ms * 1e-3) / 1e9
        knn["queries_per_s_search_kernel"] = nq / (avg_ms * 1e-3)
        knn["roofline"] = {
            "bound": "hbm", "kernel": "knn", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": load_traffic("knn", args.workload), "avg_launch_us": round(avg_ms * 1e3, 1),
            "algorithmic_bytes_per_launch": round(nq * knn_bytes_q),
            "measured_on": "overlapped step, launched per step"}
        sq = load_profile_json("knn", args.workload, "sq")
        if sq and sq.get("valu_insts_per_launch"):
            gi = sq["valu_insts_per_launch"] / (avg_ms * 1e-3) / 1e9
            knn["issue_roofline"] = {
                "bound": "alu", "kernel": "knn", "achieved": round(gi, 1),
                "peak": round(VALU_PEAK_GINST, 1), "unit": "G wave64 VALU inst/s",
                "frac": round(gi / VALU_PEAK_GINST, 4),
                "valu_insts_per_launch": sq["valu_insts_per_launch"],
                "peak_model": "256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 VALU "
                              "instruction; instructions that issue in fewer cycles take "
                              "the fraction above 1",
                "source": "profiles/knn_%s_sq.json" % args.workload}

    by_kernel = {}
    for lb, kms in kern_ms.items():
        algo = algorithmic_bytes(lb, pipe, counts, rb=rbs)
        if lb == "knn":
            algo = nq * knn_bytes_q
        if algo is None or kms <= 0:
            continue
        gbs = algo / (kms * 1e-3) / 1e9
        by_kernel[lb] = {"ms_per_step": kms, "algorithmic_mb_per_step": round(algo / 1e6, 2),
                         "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}

    line = {
        "metric": "CGA build+merge points/s & kNN queries/s at % HBM peak; learned vs binary lookup/s",
        "value": n_points / (ms_bm * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_graph, 4),
        "ms_build_merge": round(ms_bm, 4), "ms_build_merge_eager": round(ms_bm_eager, 4),
        "ms_per_step_eager": round(ms_eager, 4), "ms_per_step_serial": round(ms_serial, 4),
        "value_basis": ("points of both clouds / ms_build_merge: graph replays of the two builds "
                        "(side by side) and their merge, timed over `steps` replays; "
                        "ms_per_step is the whole step (projections, k-NN, index training and "
                        "lookups included), one graph replay per step"),
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64" if 3 * pipe.g.depth > 32 else "u32",
        "data": "synthetic",
        "config": {"workload": wl_label, "points_per_step": n_points, "queries": nq, "k": pipe.k,
                   "depth": pipe.g.depth, "projections_drop_axes": list(drops),
                   "counts": counts,
                   "sort_tuning": {k: {"radix_bits": v[0], "tile_items": v[1],
                                       "tuned_sort_ms": round(v[2], 4) if v[2] == v[2] else None}
                                   for k, v in tuned.items()},
                   "streams": "build A | build B, merge, then projections | k-NN | index "
                              "training + lookups, captured once as one HIP graph and replayed"},
        "stages": {
            "build_merge": {"ms": round(st[0], 4), "points_per_s": n_points / (st[0] * 1e-3)},
            "projections": {"ms": round(st[1], 4), "count": len(drops)},
            "knn": {"ms": round(st[2], 4), "queries_per_s": nq / (st[2] * 1e-3)},
            "index_train": {"ms": round(st[3], 4), "keys": pipe.nu},
            "learned_lookup": {"ms": round(st[4], 4), "lookups_per_s": pipe.nl / (st[4] * 1e-3)},
            "binary_lookup": {"ms": round(st[5], 4), "lookups_per_s": pipe.nl / (st[5] * 1e-3)},
        },
        "kernels_ms_per_step": kern_ms,
        "roofline": bm_roof,
        "knn": knn,
        "hbm_by_kernel": by_kernel,
        "cpu_baseline": None,
    }
    if not args.no_probe:
        progress("bandwidth probe")
        line["stream_probe"] = stream_probe(cga, device)
    if not args.no_legs or args.workload != "c2":
        progress("c2 context")
        if args.workload == "c2":
            p2, d2 = pipe, d
        else:
            p2, d2, line["c2_context"] = c2_context(cga, device, args.steps)
            p2.nu = int(p2.cnt[2].item())
        if not args.no_legs:
            progress("legs: occupancy / values / paper array ops / temporal (c2, c6)")
            line["legs"] = {"workload": WORKLOADS["c2"][0],
                            "occupancy": occupancy_codes(cga, p2),
                            "values": attribute_values(cga, p2, d2),
                            "paper_array_ops": paper_array_ops(cga, p2, d2),
                            "temporal": temporal_prediction(cga, device)}
        del p2
    if not args.no_c5:
        progress("c5 learned index vs binary search")
        line["c5"] = c5_learned_vs_binary(cga, device, args.c5_reps)
    if not args.no_c4:
        progress("c4 batched graph")
        line["c4"] = c4_batched(cga, device, args.c4_reps)
    if not args.no_cpu_baseline:
        import numpy as np
        progress("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(d, args.workload, pipe.lq.cpu().numpy().view(np.uint64))
    progress("done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
