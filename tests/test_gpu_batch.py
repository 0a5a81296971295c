"""GPU tests of the batched build + consecutive-pair merge and its graph:
every frame equals a standalone build and the oracle, every pair union
equals the oracle's, replays of the captured graph are bitwise identical to
the eager call, and no tuning changes a bit."""
import numpy as np
import pytest
import torch

import gen
import oracle
from helpers import dev, say, u32, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frames():
    # 12 LiDAR frames of a random walk, sizes log-uniform in [64, 40k], one
    # of them emptied, so the pair merges see empty operands too
    d = gen.c4_frames(seed=77, nframes=12, size_lo=64, size_hi=40_000)
    xyz, off = d["xyz"], d["off"].copy()
    keep = np.ones(len(xyz), bool)
    keep[off[5]:off[6]] = False  # frame 5 empty
    sizes = np.diff(off)
    sizes[5] = 0
    off2 = np.zeros_like(off)
    off2[1:] = np.cumsum(sizes)
    return dict(xyz=np.ascontiguousarray(xyz[keep]), off=off2, grid=d["grid"])


def _check(gpu, frames, out):
    xyz, off, g = frames["xyz"], frames["off"], frames["grid"]
    F = len(off) - 1
    ko = out.key_off.cpu().numpy()
    keys = u64(out.keys)
    cnts = u32(out.counts)
    want = []
    for f in range(F):
        wk, wc = oracle.build(xyz[off[f]:off[f + 1]], g)
        want.append(wk)
        assert np.array_equal(keys[ko[f]:ko[f + 1]], wk), f
        assert np.array_equal(cnts[ko[f]:ko[f + 1]], wc), f
    mo, mc = out.merged_off.cpu().numpy(), out.merged_cnt.cpu().numpy()
    merged = u64(out.merged)
    for f in range(F - 1):
        wm, _ = oracle.merge(want[f], want[f + 1], g.depth, g.key_mode)
        assert mc[f] == len(wm), f
        assert np.array_equal(merged[mo[f]:mo[f] + mc[f]], wm), f


def test_batch_matches_oracle(gpu, frames):
    out = gpu.cga_batch_build_merge(dev(frames["xyz"]), dev(frames["off"]), frames["grid"])
    torch.cuda.synchronize()
    _check(gpu, frames, out)


def test_batch_frame_equals_standalone_build(gpu, frames):
    xyz, off, g = frames["xyz"], frames["off"], frames["grid"]
    out = gpu.cga_batch_build_merge(dev(xyz), dev(off), g)
    for f in (0, 3, 5, 11):
        k, c = gpu.cga_build(dev(xyz[off[f]:off[f + 1]]), g)
        assert torch.equal(out.frame(f), k), f


@pytest.mark.parametrize("tune", [(4, 8), (8, 12), (11, 16), (9, 8)])
def test_batch_tunings_identical(gpu, frames, tune):
    ref = gpu.cga_batch_build_merge(dev(frames["xyz"]), dev(frames["off"]), frames["grid"])
    out = gpu.cga_batch_build_merge(dev(frames["xyz"]), dev(frames["off"]), frames["grid"],
                                    tune=tune)
    u = int(ref.key_off[-1].item())
    assert torch.equal(ref.keys[:u], out.keys[:u]) and torch.equal(ref.key_off, out.key_off)
    assert torch.equal(ref.merged_cnt, out.merged_cnt)


def test_batch_single_and_tiny(gpu):
    g = gen.Grid((0.0, 0.0, 0.0), 1.0, 6, gen.KEY_MORTON)
    rng = np.random.default_rng(5)
    for sizes in ([0], [7], [0, 0, 3], [5000, 1, 0, 4097]):
        xyz = rng.integers(0, 64, (sum(sizes), 3)).astype(np.float32)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        out = gpu.cga_batch_build_merge(dev(xyz), dev(off), g)
        _check(gpu, dict(xyz=xyz, off=off, grid=g), out)


def test_batch_segment_tile_edges(gpu):
    """Frames of exactly one tile, one tile and one key, two tiles, with
    empty frames between, under a fixed 4096-key tile (the frame-segmented
    sort): every frame sorted within its own range."""
    g = gen.Grid((0.0, 0.0, 0.0), 1.0, 10, gen.KEY_MORTON)
    rng = np.random.default_rng(11)
    sizes = [4096, 0, 4097, 8192, 1, 0, 0, 8191, 12289, 2]
    xyz = rng.integers(0, 1024, (sum(sizes), 3)).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    for tune in ((8, 16), (7, 16), (9, 32)):
        say("segmented batch sort, tune", tune)
        out = gpu.cga_batch_build_merge(dev(xyz), dev(off), g, tune=tune)
        _check(gpu, dict(xyz=xyz, off=off, grid=g), out)


def test_batch_many_frames_composite_sort(gpu):
    """Beyond 4096 frames the batch sorts the composite keys (frame bits
    included) in one sort: 4100 frames of 0 to 40 points, and 4096 frames
    (segmented) of the same points, both against the oracle."""
    g = gen.Grid((0.0, 0.0, 0.0), 1.0, 8, gen.KEY_MORTON)
    rng = np.random.default_rng(12)
    for nf in (4100, 4096):
        assert gpu.cga_batch_sort_bits(g, nf) == 24 + (13 if nf > 4096 else 0)
        sizes = rng.integers(0, 41, nf)
        sizes[rng.choice(nf, nf // 10, replace=False)] = 0
        xyz = rng.integers(0, 256, (int(sizes.sum()), 3)).astype(np.float32)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        say("batch of", nf, "frames,", len(xyz), "points")
        out = gpu.cga_batch_build_merge(dev(xyz), dev(off), g)
        _check(gpu, dict(xyz=xyz, off=off, grid=g), out)


def test_graph_replays_match_eager(gpu, frames):
    xyz, off, g = dev(frames["xyz"]), dev(frames["off"]), frames["grid"]
    ref = gpu.cga_batch_build_merge(xyz, off, g)
    torch.cuda.synchronize()
    u = int(ref.key_off[-1].item())
    graph = gpu.BatchGraph(xyz, off, g)
    for rep in range(3):
        # unrelated eager work between replays
        gpu.cga_build(xyz[:1000], g)
        graph.out.keys.fill_(0)
        graph.out.merged_cnt.fill_(-1)
        graph.launch()
        torch.cuda.synchronize()
        assert graph.status() == 0
        assert torch.equal(graph.out.key_off, ref.key_off), rep
        assert torch.equal(graph.out.keys[:u], ref.keys[:u]), rep
        assert torch.equal(graph.out.merged_cnt, ref.merged_cnt), rep
        assert torch.equal(graph.out.merged_off, ref.merged_off), rep
        # each pair's region holds merged_cnt keys; the rest of it is unused
        for f in range(len(ref.merged_cnt)):
            assert torch.equal(graph.out.pair(f), ref.pair(f)), (rep, f)
    graph.close()


def test_autotuner_choice_is_used_and_exact(gpu, frames):
    g = frames["grid"]
    rb, items, ms = gpu.cga_autotune_sort(key_bytes=8, key_bits=3 * g.depth, n=len(frames["xyz"]))
    say("autotune", rb, items, ms)
    assert 4 <= rb <= 11 and items in (8, 12, 16, 24, 32) and ms > 0
    k, c = gpu.cga_build(dev(frames["xyz"]), g)  # picks the recorded choice
    wk, wc = oracle.build(frames["xyz"], g)
    assert np.array_equal(u64(k), wk) and np.array_equal(u32(c), wc)
