"""Seeded synthetic workloads shared by the GPU path and the CPU oracle.

The paper evaluates on the 8i voxelized surface light-field sequences and the
Paris-Lille-3 LiDAR scans (Section VI-B).  Those are not available, so these
generators produce clouds of the same kind: sphere-surface and bumpy-sphere
"graphics" models and ray-cast LiDAR sweeps over a ground plane with boxes.
They return float32 xyz arrays, query points, random index sets and the grid
frame (cubic bounding box) only.  Nothing here quantizes, encodes, sorts,
merges or searches: that arithmetic belongs to the method and lives on each
side separately.

The workload recipes (sizes, distributions) are documented per function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cga_gen.c")
_LIB = os.path.join(_HERE, "libcga_gen.so")
_lib = None


def build_lib() -> str:
    """Compile the C generator core (host code only)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u64, i64, i32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.gen_spheres.argtypes = [u64, i64, i32, dbl, dbl, dbl, dbl, dbl, P, P]
        lib.gen_uniform_box.argtypes = [u64, u64, i64, P, P, P]
        lib.gen_bumpy_sphere.argtypes = [u64, i64, i32, dbl, P, P]
        lib.gen_lidar_scene.argtypes = [u64, i32, dbl, dbl, dbl, P]
        lib.gen_lidar_sweep.argtypes = [u64, u64, P, i32, P, dbl, i32, i64, dbl, dbl, dbl, P]
        lib.gen_random_walk.argtypes = [u64, i32, P, dbl, dbl, dbl, dbl, P, P]
        lib.gen_jittered_picks.argtypes = [u64, u64, P, i64, i64, dbl, P]
        lib.gen_uniform_index.argtypes = [u64, u64, i64, u64, P]
        lib.gen_uniform_u64.argtypes = [u64, u64, i64, u64, u64, P]
        lib.gen_subset.argtypes = [u64, i64, i64, P]
        lib.gen_subset.restype = i64
        lib.gen_shuffle_i64.argtypes = [u64, i64, P]
        lib.gen_raw.argtypes = [u64, u64, u64, i32, P]
        lib.gen_attributes.argtypes = [u64, u64, i64, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Grid frame
# --------------------------------------------------------------------------
KEY_MORTON = 0
KEY_LINEAR = 1


@dataclass(frozen=True)
class Grid:
    """Quantization frame: voxel = floor((p - origin) * scale), per axis,
    clamped to [0, 2^depth - 1]; keys in MORTON or LINEAR order."""
    origin: tuple  # three float32 values
    scale: float   # float32 value
    depth: int
    key_mode: int = KEY_MORTON

    def with_mode(self, key_mode: int) -> "Grid":
        return Grid(self.origin, self.scale, self.depth, key_mode)


def cubic_grid(clouds, depth: int, key_mode: int = KEY_MORTON) -> Grid:
    """Cubic bounding box over every cloud that will be combined (the root box
    of Section II-E's bounding-box alignment), mapped onto 2^depth voxels per
    axis.  Origin and scale are rounded to float32 once."""
    lo = np.full(3, np.inf)
    hi = np.full(3, -np.inf)
    for c in clouds:
        if len(c):
            c64 = c.astype(np.float64)
            lo = np.minimum(lo, c64.min(axis=0))
            hi = np.maximum(hi, c64.max(axis=0))
    ext = float(np.max(hi - lo))
    if not np.isfinite(ext) or ext <= 0:
        ext = 1.0
    scale = np.float32((2.0 ** depth) / (ext * (1.0 + 2.0 ** -20)))
    origin = tuple(float(np.float32(v)) for v in lo)
    return Grid(origin, float(scale), depth, key_mode)


# --------------------------------------------------------------------------
# Raw generators
# --------------------------------------------------------------------------
def spheres(seed: int, n: int, nsph: int = 8, jitter: float = 1e-3, rot_deg: float = 0.0,
            pivot=(0.5, 0.5), shift_x: float = 0.0, with_copy: bool = False):
    lib = _load()
    a = np.empty((n, 3), np.float32)
    b = np.empty((n, 3), np.float32) if with_copy else None
    lib.gen_spheres(seed, n, nsph, jitter, rot_deg, pivot[0], pivot[1], shift_x, _p(a),
                    _p(b) if b is not None else None)
    return (a, b) if with_copy else a


def uniform_box(seed: int, stream: int, n: int, lo, hi) -> np.ndarray:
    lib = _load()
    out = np.empty((n, 3), np.float32)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    lib.gen_uniform_box(seed, stream, n, _p(lo), _p(hi), _p(out))
    return out


def bumpy_sphere(seed: int, n: int, nbumps: int = 64, rot_deg: float = 0.0, with_copy=False):
    lib = _load()
    a = np.empty((n, 3), np.float32)
    b = np.empty((n, 3), np.float32) if with_copy else None
    lib.gen_bumpy_sphere(seed, n, nbumps, rot_deg, _p(a), _p(b) if b is not None else None)
    return (a, b) if with_copy else a


def lidar_scene(seed: int, nboxes: int = 200, half_extent: float = 50.0,
                clear_x=(0.0, 0.5)) -> np.ndarray:
    lib = _load()
    boxes = np.empty((nboxes, 6), np.float64)
    lib.gen_lidar_scene(seed, nboxes, half_extent, clear_x[0], clear_x[1], _p(boxes))
    return boxes


def lidar_sweep(seed: int, stream: int, boxes: np.ndarray, pose, yaw_deg: float = 0.0,
                rings: int = 64, naz: int = 16384, el=(-24.0, -2.0),
                sigma: float = 0.02) -> np.ndarray:
    lib = _load()
    out = np.empty((rings * naz, 3), np.float32)
    pose = np.asarray(pose, np.float64)
    boxes = np.ascontiguousarray(boxes, np.float64)
    lib.gen_lidar_sweep(seed, stream, _p(boxes), len(boxes), _p(pose), yaw_deg, rings, naz,
                        el[0], el[1], sigma, _p(out))
    return out


def random_walk(seed: int, nframes: int, start=(0.0, 0.0, 1.8), step: float = 0.2,
                yaw_step: float = 1.0, size_lo: float = 1e4, size_hi: float = 2e6):
    lib = _load()
    poses = np.empty((nframes, 4), np.float64)
    sizes = np.empty(nframes, np.int64)
    st = np.asarray(start, np.float64)
    lib.gen_random_walk(seed, nframes, _p(st), step, yaw_step, size_lo, size_hi, _p(poses),
                        _p(sizes))
    return poses, sizes


def jittered_picks(seed: int, stream: int, src: np.ndarray, n: int, sigma: float) -> np.ndarray:
    lib = _load()
    src = np.ascontiguousarray(src, np.float32)
    out = np.empty((n, 3), np.float32)
    lib.gen_jittered_picks(seed, stream, _p(src), len(src), n, sigma, _p(out))
    return out


def uniform_index(seed: int, stream: int, n: int, m: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, np.int64)
    lib.gen_uniform_index(seed, stream, n, m, _p(out))
    return out


def uniform_u64(seed: int, stream: int, n: int, lo: int, hi: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, np.uint64)
    lib.gen_uniform_u64(seed, stream, n, lo, hi, _p(out))
    return out


def subset(seed: int, u: int, m: int) -> np.ndarray:
    lib = _load()
    out = np.empty(min(u, m), np.int64)
    k = lib.gen_subset(seed, u, m, _p(out))
    return out[:k]


def shuffle(seed: int, a: np.ndarray) -> np.ndarray:
    lib = _load()
    a = np.ascontiguousarray(a, np.int64).copy()
    lib.gen_shuffle_i64(seed, len(a), _p(a))
    return a


def attributes(seed: int, stream: int, n: int) -> np.ndarray:
    """Seeded per-point attributes: four 8-bit channels packed in uint32
    (channel c in bits 8c .. 8c + 7), e.g. RGB plus one spare channel."""
    lib = _load()
    out = np.empty(n, np.uint32)
    lib.gen_attributes(seed, stream, n, _p(out))
    return out


def raw(seed: int, stream: int, index: int, n: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, np.uint64)
    lib.gen_raw(seed, stream, index, n, _p(out))
    return out


# --------------------------------------------------------------------------
# Workloads.  Each returns a dict of numpy arrays plus the Grid.
# --------------------------------------------------------------------------
def c1_spheres(seed: int = 1001, n: int = 100_000, nq: int = 1000) -> dict:
    """100k points on 8 random spheres in the unit cube with N(0, 1e-3) jitter;
    a copy rotated 5 degrees about z through (0.5, 0.5) and shifted +0.01 in x;
    nq uniform queries in [0,1)^3.  Grid: origin 0, scale 1024, depth 10 (exact
    power-of-two quantization), 30-bit Morton keys in uint32."""
    a, b = spheres(seed, n, 8, 1e-3, 5.0, (0.5, 0.5), 0.01, with_copy=True)
    q = uniform_box(seed, 3, nq, (0, 0, 0), (1, 1, 1))
    grid = Grid((0.0, 0.0, 0.0), 1024.0, 10, KEY_MORTON)
    return dict(a=a, b=b, q=q, grid=grid, k=1)


def c2_lidar(seed: int = 1002, rings: int = 64, naz: int = 16384, nq: int = 100_000,
             depth: int = 12) -> dict:
    """Two LiDAR sweeps (64 rings x 16384 azimuths = 1,048,576 points each) of a
    ground plane plus 200 boxes in a 100 m square, sensors at (0,0,1.8) and
    (0.5,0,1.8), range noise N(0, 0.02 m); nq queries = points of sweep A plus
    N(0, 0.1 m) offsets; k = 8.  Grid: cubic bbox of both sweeps and the
    queries, depth 12, Morton keys in uint64."""
    boxes = lidar_scene(seed)
    a = lidar_sweep(seed, 1, boxes, (0.0, 0.0, 1.8), 0.0, rings, naz)
    b = lidar_sweep(seed, 2, boxes, (0.5, 0.0, 1.8), 0.0, rings, naz)
    q = jittered_picks(seed, 3, a, nq, 0.1)
    grid = cubic_grid([a, b, q], depth)
    return dict(a=a, b=b, q=q, grid=grid, k=8)


def c3_bumpy(seed: int = 1003, n: int = 10_000_000, nq: int = 1_000_000,
             depth: int = 14) -> dict:
    """10M points on a unit sphere perturbed by 64 Gaussian bumps (amplitude
    U[0,0.1], width U[0.05,0.3]); a copy rotated 10 degrees about z; nq
    queries uniform in the merged bounding box; k = 16.  Grid: cubic bbox,
    depth 14, 42-bit Morton keys in uint64."""
    a, b = bumpy_sphere(seed, n, 64, 10.0, with_copy=True)
    lo = np.minimum(a.min(0), b.min(0)).astype(np.float64)
    hi = np.maximum(a.max(0), b.max(0)).astype(np.float64)
    q = uniform_box(seed, 3, nq, lo, hi)
    grid = cubic_grid([a, b], depth)
    return dict(a=a, b=b, q=q, grid=grid, k=16)


def c6_frames(seed: int = 1006, n: int = 1_000_000, depth: int = 10) -> dict:
    """A reference and a predicted frame of a moving object, standing in for
    the voxelized full-body sequences that point cloud compression is
    evaluated on (about 10^6 points on a 1024^3 grid per frame): a bumpy
    sphere of n points squeezed to a standing figure's proportions (0.35 :
    1 : 0.2); the predicted frame moves the object by an offset of -3 .. 3
    voxels per axis, each octant (about the centre) by a further -1 .. 1, and
    draws 2 % of its points afresh.  Colours (RGB + 255, packed as the Value array
    packs them) are a smooth field of each point's position before the motion
    plus N(0, 2) noise per channel and frame.  LINEAR cubic grid of the
    given depth over the object grown by 2 % (room for the motion)."""
    rng = np.random.default_rng(seed)
    shape = np.array([0.35, 1.0, 0.2], np.float32)  # a standing figure's proportions
    ref = bumpy_sphere(seed, n) * shape
    grid = cubic_grid([ref * np.float32(1.02)], depth, KEY_LINEAR)
    voxel = 1.0 / grid.scale
    octant = ((ref[:, 0] > 0).astype(np.int64) << 2) | ((ref[:, 1] > 0).astype(np.int64) << 1) | (
        ref[:, 2] > 0).astype(np.int64)
    offsets = rng.integers(-3, 4, (1, 3)) + rng.integers(-1, 2, (8, 3))
    pred = (ref.astype(np.float64) + offsets[octant] * voxel).astype(np.float32)
    fresh = rng.random(n) < 0.02
    pred[fresh] = bumpy_sphere(seed + 1, int(fresh.sum())) * shape
    base = np.stack([np.sin(3.0 * ref[:, 0]), np.sin(3.0 * ref[:, 1] + 1.0),
                     np.sin(3.0 * ref[:, 2] + 2.0)], 1) * 100.0 + 128.0

    def colours(noise):
        c = np.clip(np.rint(base + noise), 0, 255).astype(np.uint32)
        return c[:, 0] | (c[:, 1] << 8) | (c[:, 2] << 16) | np.uint32(255 << 24)

    return dict(ref=ref, pred=pred, ref_values=colours(rng.normal(0, 2, (n, 3))),
                pred_values=colours(rng.normal(0, 2, (n, 3))), offsets=offsets, grid=grid)


def c4_frames(seed: int = 1004, nframes: int = 256, size_lo: float = 1e4,
              size_hi: float = 2e6, depth: int = 12) -> dict:
    """nframes LiDAR frames of the two-sweep scene, sensed from a random walk
    (0.2 m per frame in a uniform heading, yaw U[-1,1] degrees per frame);
    frame sizes log-uniform in [size_lo, size_hi] realised as 64 rings x
    round(n_f/64) azimuths.  One shared cubic grid, depth 12, uint64 keys."""
    boxes = lidar_scene(seed)
    poses, sizes = random_walk(seed, nframes, (0.0, 0.0, 1.8), 0.2, 1.0, size_lo, size_hi)
    frames = []
    for f in range(nframes):
        naz = max(1, int(round(sizes[f] / 64)))
        frames.append(lidar_sweep(seed, 100 + f, boxes, poses[f, :3], poses[f, 3], 64, naz))
    off = np.zeros(nframes + 1, np.int64)
    off[1:] = np.cumsum([len(x) for x in frames])
    xyz = np.concatenate(frames, axis=0)
    grid = cubic_grid([xyz], depth)
    return dict(xyz=xyz, off=off, grid=grid)


def c5_sweeps(seed: int = 1005, nsweeps: int = 52, naz: int = 16384, depth: int = 16) -> dict:
    """Point source of the learned-index key arrays: nsweeps LiDAR sweeps of
    the two-sweep scene from random-walk poses, with a cubic grid at depth 16
    (48-bit Morton keys).  The sorted unique keys built from these points are
    subsampled to exactly 50M with `subset`."""
    boxes = lidar_scene(seed)
    poses, _ = random_walk(seed, nsweeps, (0.0, 0.0, 1.8), 0.2, 1.0)
    sw = [lidar_sweep(seed, 100 + f, boxes, poses[f, :3], poses[f, 3], 64, naz)
          for f in range(nsweeps)]
    xyz = np.concatenate(sw, axis=0)
    grid = cubic_grid([xyz], depth)
    return dict(xyz=xyz, grid=grid)


def lookup_queries(seed: int, keys: np.ndarray, nq: int) -> np.ndarray:
    """nq lookup queries over a sorted key array: half are keys picked at
    uniform random positions, half are uniform u64 values in [keys[0],
    keys[-1]] (absent with overwhelming probability for sparse keys); shuffled."""
    n_present = nq // 2
    idx = uniform_index(seed, 21, n_present, len(keys))
    present = keys[idx]
    absent = uniform_u64(seed, 22, nq - n_present, int(keys[0]), int(keys[-1]))
    q = np.concatenate([present.astype(np.uint64), absent])
    perm = shuffle(seed, np.arange(nq, dtype=np.int64))
    return q[perm]
