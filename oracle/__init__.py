"""CGA oracle -- TEST INFRASTRUCTURE ONLY.

Python access to the plain CPU oracle in ``cga_oracle.cpp``.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package; the product library never does.  Every function returns numpy
arrays; keys are always handled as uint64 here.

Each wrapper names the passage of the paper that its C function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cga_oracle.cpp")
_LIB = os.path.join(_HERE, "libcga_oracle.so")
_lib = None

MORTON = 0
LINEAR = 1


def build_lib() -> str:
    tmp = _LIB + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u32, i32, f32 = ctypes.c_int64, ctypes.c_uint32, ctypes.c_int, ctypes.c_float
        lib.or_quantize.argtypes = [P, i64, P, f32, u32, P]
        lib.or_quantize.restype = i32
        lib.or_encode.argtypes = [P, i64, u32, i32, P]
        lib.or_decode.argtypes = [P, i64, u32, i32, P]
        lib.or_encode2.argtypes = [P, P, i64, u32, i32, P]
        lib.or_build.argtypes = [P, i64, P, f32, u32, i32, P, P]
        lib.or_build.restype = i64
        lib.or_arrays.argtypes = [P, i64, u32, i32, P, P, P, P, P, P, P, P]
        lib.or_merge.argtypes = [P, i64, P, i64, u32, i32, P, P]
        lib.or_merge.restype = i64
        lib.or_project.argtypes = [P, i64, u32, i32, i32, P, P]
        lib.or_project.restype = i64
        lib.or_knn_brute.argtypes = [P, i64, u32, i32, P, i64, P, f32, i32, P, P]
        lib.or_knn_brute.restype = i32
        lib.or_knn_kdtree.argtypes = [P, i64, u32, i32, P, i64, P, f32, i32, P, P]
        lib.or_knn_kdtree.restype = i32
        lib.or_nn_cga.argtypes = [P, i64, P, P, P, P, u32, i32, P, i64, P, P]
        lib.or_lower_bound.argtypes = [P, i64, P, i64, P, P]
        lib.or_lookup_cga.argtypes = [P, i64, P, P, P, P, P, i64, P]
        lib.or_temporal_predict.argtypes = [P, P, i64, P, P, i64, u32, i32, i32, i32, P, P, P,
                                            P, P, P, P, P]
        lib.or_mlp_loss_grad.argtypes = [P, P, P, i64, P, P]
        lib.or_occupancy.argtypes = [P, i64, u32, P, P]
        lib.or_voxel_values.argtypes = [P, i64, P, P, f32, u32, i32, P, P]
        lib.or_voxel_values.restype = i64
        lib.or_merge_values.argtypes = [P, P, i64, P, P, i64, i32, P, P]
        lib.or_merge_values.restype = i64
        lib.or_occupancy.restype = i64
        lib.or_mlp_loss_grad.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _u64(a):
    return np.ascontiguousarray(a, np.uint64)


def _origin(grid):
    return np.asarray(grid.origin, np.float32)


class NonFinite(ValueError):
    pass


# ---------------------------------------------------------------- grid, keys
def quantize(xyz, grid) -> np.ndarray:
    """Grid rule (Section II-E bounding box; Table II integer voxels)."""
    xyz = _f32(xyz).reshape(-1, 3)
    vox = np.empty_like(xyz, dtype=np.uint32)
    if _load().or_quantize(_p(xyz), len(xyz), _p(_origin(grid)), grid.scale, grid.depth, _p(vox)):
        raise NonFinite("non-finite coordinate")
    return vox


def encode(vox, depth: int, mode: int) -> np.ndarray:
    vox = np.ascontiguousarray(vox, np.uint32).reshape(-1, 3)
    out = np.empty(len(vox), np.uint64)
    _load().or_encode(_p(vox), len(vox), depth, mode, _p(out))
    return out


def decode(keys, depth: int, mode: int) -> np.ndarray:
    keys = _u64(keys)
    out = np.empty((len(keys), 3), np.uint32)
    _load().or_decode(_p(keys), len(keys), depth, mode, _p(out))
    return out


def encode2(u, v, depth: int, mode: int) -> np.ndarray:
    u = np.ascontiguousarray(u, np.uint32)
    v = np.ascontiguousarray(v, np.uint32)
    out = np.empty(len(u), np.uint64)
    _load().or_encode2(_p(u), _p(v), len(u), depth, mode, _p(out))
    return out


# ---------------------------------------------------------------- operations
def build(xyz, grid):
    """CGA construction (Section V): (sorted unique keys, points per voxel)."""
    xyz = _f32(xyz).reshape(-1, 3)
    keys = np.empty(len(xyz), np.uint64)
    counts = np.empty(len(xyz), np.uint32)
    u = _load().or_build(_p(xyz), len(xyz), _p(_origin(grid)), grid.scale, grid.depth,
                         grid.key_mode, _p(keys), _p(counts))
    if u < 0:
        raise NonFinite("non-finite coordinate")
    return keys[:u].copy(), counts[:u].copy()


def arrays(keys, depth: int, mode: int) -> dict:
    """The paper's X_index, X_pointer, Y_index, Y_pointer, Z_index (Section V)."""
    keys = _u64(keys)
    n = len(keys)
    xi = np.empty(max(n, 1), np.uint32)
    xp = np.empty(n + 1, np.int64)
    yi = np.empty(max(n, 1), np.uint32)
    yp = np.empty(n + 1, np.int64)
    zi = np.empty(max(n, 1), np.uint32)
    nx, nxy, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _load().or_arrays(_p(keys), n, depth, mode, _p(xi), _p(xp), _p(yi), _p(yp), _p(zi),
                      ctypes.byref(nx), ctypes.byref(nxy), ctypes.byref(nz))
    nx, nxy, nz = nx.value, nxy.value, nz.value
    return dict(x_index=xi[:nx].copy(), x_pointer=xp[:nx + 1].copy(), y_index=yi[:nxy].copy(),
                y_pointer=yp[:nxy + 1].copy(), z_index=zi[:nz].copy())


def merge(a, b, depth: int, mode: int):
    """Merge, Eq. (1): (union keys, provenance 1=A 2=B 3=both)."""
    a, b = _u64(a), _u64(b)
    out = np.empty(len(a) + len(b), np.uint64)
    src = np.empty(len(a) + len(b), np.uint8)
    n = _load().or_merge(_p(a), len(a), _p(b), len(b), depth, mode, _p(out), _p(src))
    return out[:n].copy(), src[:n].copy()


def project(keys, depth: int, mode: int, drop_axis: int):
    """Orthogonal projection, Eq. (3) with m = 1: (2D keys, voxels per pixel)."""
    keys = _u64(keys)
    out = np.empty(len(keys), np.uint64)
    cnt = np.empty(len(keys), np.uint32)
    n = _load().or_project(_p(keys), len(keys), depth, mode, drop_axis, _p(out), _p(cnt))
    return out[:n].copy(), cnt[:n].copy()


def _knn(fn, keys, queries, grid, k):
    keys = _u64(keys)
    q = _f32(queries).reshape(-1, 3)
    idx = np.empty((len(q), k), np.int64)
    d2 = np.empty((len(q), k), np.uint64)
    rc = fn(_p(keys), len(keys), grid.depth, grid.key_mode, _p(q), len(q), _p(_origin(grid)),
            grid.scale, k, _p(idx), _p(d2))
    if rc:
        raise NonFinite("non-finite query")
    return idx, d2


def knn_brute(keys, queries, grid, k: int):
    """k-NN by definition, Eq. (7)-(8), ties by key: (index, squared distance)."""
    return _knn(_load().or_knn_brute, keys, queries, grid, k)


def knn_kdtree(keys, queries, grid, k: int):
    """kd-tree k-NN after Algorithm 1, exact with ties by key."""
    return _knn(_load().or_knn_kdtree, keys, queries, grid, k)


def nn_cga(arr: dict, qvox, depth: int, mode: int):
    """The paper's CGA nearest-neighbour search (Section V-C), 1-NN, on the five
    arrays; returns (position in Z_index order, squared distance)."""
    qvox = np.ascontiguousarray(qvox, np.uint32).reshape(-1, 3)
    pos = np.empty(len(qvox), np.int64)
    d2 = np.empty(len(qvox), np.uint64)
    xi = np.ascontiguousarray(arr["x_index"], np.uint32)
    xp = np.ascontiguousarray(arr["x_pointer"], np.int64)
    yi = np.ascontiguousarray(arr["y_index"], np.uint32)
    yp = np.ascontiguousarray(arr["y_pointer"], np.int64)
    zi = np.ascontiguousarray(arr["z_index"], np.uint32)
    _load().or_nn_cga(_p(xi), len(xi), _p(xp), _p(yi), _p(yp), _p(zi), depth, mode, _p(qvox),
                      len(qvox), _p(pos), _p(d2))
    return pos, d2


def lookup_cga(arr: dict, qvox):
    """Point lookup on the five arrays (Section V-A, three-level search):
    position in Z_index order, -1 when absent."""
    qvox = np.ascontiguousarray(qvox, np.uint32).reshape(-1, 3)
    pos = np.empty(len(qvox), np.int64)
    xi = np.ascontiguousarray(arr["x_index"], np.uint32)
    xp = np.ascontiguousarray(arr["x_pointer"], np.int64)
    yi = np.ascontiguousarray(arr["y_index"], np.uint32)
    yp = np.ascontiguousarray(arr["y_pointer"], np.int64)
    zi = np.ascontiguousarray(arr["z_index"], np.uint32)
    _load().or_lookup_cga(_p(xi), len(xi), _p(xp), _p(yi), _p(yp), _p(zi), _p(qvox), len(qvox),
                          _p(pos))
    return pos


def temporal_predict(ref_keys, ref_vals, pred_keys, pred_vals, depth: int, mode: int,
                     window: int = 2, max_iter: int = 20) -> dict:
    """Temporal prediction of a frame from a reference frame (Section V-D):
    8-centre k-means of both frames from the bounding-box corners, motion
    vectors from corresponding centroids, SAD matching of every motion-
    compensated predicted voxel in a +-window box of the reference, residual."""
    rk, pk = _u64(ref_keys), _u64(pred_keys)
    rv = np.ascontiguousarray(ref_vals, np.uint32)
    pv = np.ascontiguousarray(pred_vals, np.uint32)
    nr, npred = len(rk), len(pk)
    out = dict(ref_assign=np.empty(max(nr, 1), np.uint8), pred_assign=np.empty(max(npred, 1), np.uint8),
               centroids=np.empty((2, 8, 3), np.float64), mv=np.empty((8, 3), np.int32),
               iters=np.empty(2, np.int32), match=np.empty(max(npred, 1), np.int64),
               sad=np.empty(max(npred, 1), np.uint32), residual=np.empty((max(npred, 1), 4), np.int16))
    _load().or_temporal_predict(_p(rk), _p(rv), nr, _p(pk), _p(pv), npred, depth, mode, window,
                                max_iter, _p(out["ref_assign"]), _p(out["pred_assign"]),
                                _p(out["centroids"]), _p(out["mv"]), _p(out["iters"]),
                                _p(out["match"]), _p(out["sad"]), _p(out["residual"]))
    for name, n in (("ref_assign", nr), ("pred_assign", npred), ("match", npred), ("sad", npred),
                    ("residual", npred)):
        out[name] = out[name][:n].copy()
    return out


def lower_bound(keys, q):
    """rank = lower_bound(keys, q); found = keys[rank] == q."""
    keys, q = _u64(keys), _u64(q)
    rank = np.empty(len(q), np.int64)
    found = np.empty(len(q), np.uint8)
    _load().or_lower_bound(_p(keys), len(keys), _p(q), len(q), _p(rank), _p(found))
    return rank, found


def voxel_values(xyz, attr, grid):
    """Value array (Section V): (keys, per-voxel channel-wise average of the
    points' packed 4 x 8-bit values, rounded half up)."""
    xyz = _f32(xyz)
    attr = np.ascontiguousarray(attr, np.uint32)
    keys = np.empty(len(xyz), np.uint64)
    vals = np.empty(len(xyz), np.uint32)
    u = _load().or_voxel_values(_p(xyz), len(xyz), _p(attr), _p(_origin(grid)), grid.scale,
                                grid.depth, grid.key_mode, _p(keys), _p(vals))
    if u < 0:
        raise NonFinite("non-finite coordinate")
    return keys[:u].copy(), vals[:u].copy()


BASE, AVERAGE = 0, 1


def merge_values(ka, va, kb, vb, policy: int):
    """Merge with values (Eq. (1), Section II-A): (union keys, values) with the
    base's (a's) value or the rounded channel average on overlapping voxels."""
    ka, kb = _u64(ka), _u64(kb)
    va = np.ascontiguousarray(va, np.uint32)
    vb = np.ascontiguousarray(vb, np.uint32)
    keys = np.empty(len(ka) + len(kb), np.uint64)
    vals = np.empty(len(ka) + len(kb), np.uint32)
    u = _load().or_merge_values(_p(ka), _p(va), len(ka), _p(kb), _p(vb), len(kb), policy,
                                _p(keys), _p(vals))
    return keys[:u].copy(), vals[:u].copy()


def occupancy(keys, depth: int):
    """Octree occupancy codes (Section II-E, constructing the octree / coding of
    the occupancy codes) of a sorted unique MORTON key set: (codes root first,
    level by level, cells in key order; occupied cells per level, index L)."""
    keys = _u64(keys)
    occ = np.empty(max(1, len(keys) * depth), np.uint8)
    counts = np.empty(depth + 1, np.int64)
    t = _load().or_occupancy(_p(keys), len(keys), depth, _p(occ), _p(counts))
    return occ[:t].copy(), counts


def mlp_loss_grad(params, x, t):
    """fp64 loss and analytic gradient of the 1-16-1 ReLU leaf network under
    mean squared error; parameter order w1[16], b1[16], w2[16], b2."""
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    g = np.empty(49, np.float64)
    kink = ctypes.c_int64()
    loss = _load().or_mlp_loss_grad(_p(p), _p(x), _p(t), len(x), _p(g), ctypes.byref(kink))
    return loss, g, kink.value
