"""Python binding of libcga.so, the MI355X compressed-geometric-array library.

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and the stream.  Function names
match the C entry points of include/cga.h.  Keys travel as int32 / int64
tensors holding the uint32 / uint64 bit patterns.

The library must be built (``python -m paper_2110_11616_amd._build`` or
``__graft_entry__.build()``); importing without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcga.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2110_11616_amd._build.build()")

lib = ctypes.CDLL(LIB_PATH)

KEY_MORTON = 0
KEY_LINEAR = 1

OK, EINVAL, ECAPACITY, EMISMATCH, ENONFINITE, EHIP, EWORKSPACE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7


class cga_grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("scale", ctypes.c_float),
                ("depth", ctypes.c_uint32), ("key_mode", ctypes.c_uint32)]


class cga_tune(ctypes.Structure):
    _fields_ = [("radix_bits", ctypes.c_uint32), ("tile_items", ctypes.c_uint32)]


class CgaError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.cga_strerror(status).decode()
        if status == EHIP:
            msg += f" (hipError {lib.cga_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")
        self.status = status


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_GP = ctypes.POINTER(cga_grid)
_TP = ctypes.POINTER(cga_tune)
_I64P = ctypes.POINTER(ctypes.c_int64)


def _sig(name, restype, *args):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = list(args)
    return f


_sig("cga_strerror", ctypes.c_char_p, ctypes.c_int)
_sig("cga_last_hip_error", ctypes.c_int)
_sig("cga_key_bytes", _SZ, _GP)
_sig("cga_key2_bytes", _SZ, _GP)
_sig("cga_ws_status", ctypes.c_int, _P, _P)
_sig("cga_build_workspace_bytes", _SZ, _GP, _I64)
_sig("cga_build", ctypes.c_int, _GP, _P, _I64, _P, _P, _I64, _P, _I64P, _P, _SZ, _TP, _P)
_sig("cga_encode_keys", ctypes.c_int, _GP, _P, _I64, _P, _P, _SZ, _P)
_sig("cga_sort_workspace_bytes", _SZ, _GP, _I64)
_sig("cga_sort_keys", ctypes.c_int, _GP, _P, _I64, _P, ctypes.c_uint32, _P, _P, _SZ, _TP, _P)
_sig("cga_to_arrays_workspace_bytes", _SZ, _GP, _I64)
_sig("cga_to_arrays", ctypes.c_int, _GP, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _I64P, _I64P,
     _P, _SZ, _P)
_sig("cga_arrays_ops_workspace_bytes", _SZ)
_sig("cga_arrays_lookup", ctypes.c_int, _GP, _P, _I64, _P, _P, _P, _I64, _P, _P, _P, _I64, _P,
     _I64, _P, _P, _SZ, _P)
_sig("cga_arrays_nn", ctypes.c_int, _GP, _P, _I64, _P, _P, _P, _I64, _P, _P, _P, _I64, _P, _I64,
     _P, _P, _P, _SZ, _P)
_sig("cga_temporal_workspace_bytes", _SZ)
_sig("cga_temporal_predict", ctypes.c_int, _GP, _P, _P, _I64, _P, _P, _I64, ctypes.c_int,
     ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P)
_sig("cga_merge_workspace_bytes", _SZ, _GP, _I64, _I64)
_sig("cga_merge", ctypes.c_int, _GP, _P, _I64, _P, _P, _I64, _P, _P, _P, _I64, _P, _I64P, _P, _SZ,
     _P)
_sig("cga_merge_noalloc", ctypes.c_int, _GP, _P, _I64, _P, _P, _I64, _P, _P, _P, _I64, _P, _I64P,
     _P)
MERGE_NOALLOC_MAX_KEYS = 1 << 28
_sig("cga_project_workspace_bytes", _SZ, _GP, _I64)
_sig("cga_project", ctypes.c_int, _GP, _P, _I64, _P, ctypes.c_int, _P, _P, _I64, _P, _I64P, _P,
     _SZ, _TP, _P)
_sig("cga_knn_workspace_bytes", _SZ, _GP, _I64, _I64)
_sig("cga_knn", ctypes.c_int, _GP, _P, _I64, _P, _P, _I64, ctypes.c_int, _P, _P, _P, _SZ, _P)
_sig("cga_knn_count", ctypes.c_int, _GP, _P, _I64, _P, _P, _I64, ctypes.c_int, _P, _P, _P, _P, _SZ,
     _P)
_sig("cga_binary_lookup", ctypes.c_int, _P, _I64, _P, _P, _I64, _P, _P, _P)


class cga_index_params(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_uint32), ("leaf_kind", ctypes.c_uint32),
                ("epochs", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("root_segments", ctypes.c_uint32)]


_IPP = ctypes.POINTER(cga_index_params)
_sig("cga_index_bytes", _SZ, _IPP)
_sig("cga_index_train_workspace_bytes", _SZ, _IPP, _I64)
_sig("cga_index_train", ctypes.c_int, _P, _I64, _IPP, _P, _SZ, _P, _SZ, _P)
_sig("cga_index_lookup_workspace_bytes", _SZ)
_sig("cga_index_lookup", ctypes.c_int, _P, _P, _I64, _P, _I64, _P, _P, _P, _P, _SZ, _P)
_sig("cga_index_stats", ctypes.c_int, _P, _P, _P, _P)
_sig("cga_mlp_loss_grad", ctypes.c_int, _P, _P, _P, _I64, _P, _P, _P)
_sig("cga_batch_workspace_bytes", _SZ, _GP, ctypes.c_int, _I64)
_sig("cga_batch_sort_bits", ctypes.c_int, _GP, ctypes.c_int)
_sig("cga_batch_build_merge", ctypes.c_int, _GP, _P, _P, ctypes.c_int, _I64, _P, _P, _P, _P, _P, _P,
     _TP, _P, _SZ, _P)
_sig("cga_batch_graph_create", ctypes.c_int, _GP, _P, _P, ctypes.c_int, _I64, _P, _P, _P, _P, _P,
     _P, _TP, _P, _SZ, ctypes.POINTER(ctypes.c_void_p))
_sig("cga_batch_graph_launch", ctypes.c_int, _P, _P)
_sig("cga_batch_graph_destroy", ctypes.c_int, _P)
_sig("cga_autotune_workspace_bytes", _SZ, ctypes.c_uint32, _I64)
_sig("cga_autotune_sort", ctypes.c_int, _P, ctypes.c_uint32, ctypes.c_uint32, _I64, _P, _SZ, _TP,
     ctypes.POINTER(ctypes.c_float), _P)
_sig("cga_voxel_values_workspace_bytes", _SZ, _GP, _I64)
_sig("cga_voxel_values", ctypes.c_int, _GP, _P, _I64, _P, _P, _I64, _P, _P, _P, _SZ, _P)
_sig("cga_merge_values_workspace_bytes", _SZ)
_sig("cga_merge_values", ctypes.c_int, _GP, _P, _P, _I64, _P, _P, _P, _I64, _P, _P, _I64, _P,
     ctypes.c_int, _P, _P, _SZ, _P)
_sig("cga_occupancy_workspace_bytes", _SZ, _GP, _I64)
_sig("cga_occupancy", ctypes.c_int, _GP, _P, _I64, _P, _P, _I64, _P, _P, _SZ, _P)
_sig("cga_prof_enable", ctypes.c_int, ctypes.c_char_p)
_sig("cga_prof_disable", ctypes.c_int)
_sig("cga_prof_reset", ctypes.c_int)
_sig("cga_prof_read", ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), _I64P)
_sig("cga_stream_probe", ctypes.c_int, _P, _P, _SZ, ctypes.c_int, ctypes.c_int, _P)


# ------------------------------------------------------------------ helpers
@dataclass(frozen=True)
class Grid:
    origin: tuple
    scale: float
    depth: int
    key_mode: int = KEY_MORTON


def grid_struct(g) -> cga_grid:
    s = cga_grid()
    for a in range(3):
        s.origin[a] = float(g.origin[a])
    s.scale = float(g.scale)
    s.depth = int(g.depth)
    s.key_mode = int(g.key_mode)
    return s


def tune_struct(t):
    if t is None:
        return None
    s = cga_tune()
    s.radix_bits, s.tile_items = int(t[0]), int(t[1])
    return ctypes.byref(s)


def key_dtype(g) -> torch.dtype:
    return torch.int64 if 3 * g.depth > 32 else torch.int32


def key2_dtype(g) -> torch.dtype:
    return torch.int64 if 2 * g.depth > 32 else torch.int32


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc: int, where: str):
    if rc != OK:
        raise CgaError(rc, where)


class Workspaces:
    """Reusable device workspaces, grown on demand, one per name."""

    def __init__(self, device="cuda"):
        self.device = device
        self.bufs = {}

    def get(self, name: str, nbytes: int) -> torch.Tensor:
        b = self.bufs.get(name)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self.bufs[name] = b
        return b


_default_ws = None


def _ws(name, nbytes, ws):
    global _default_ws
    if ws is None:
        if _default_ws is None:
            _default_ws = Workspaces()
        ws = _default_ws
    return ws.get(name, nbytes)


def _cap_tensor(n, dtype, device):
    return torch.empty(max(int(n), 1), dtype=dtype, device=device)


def _hostcount():
    return ctypes.c_int64(0)


# --------------------------------------------------------------- entry points
def cga_build(xyz: torch.Tensor, grid, *, counts: bool = True, cap=None, tune=None, keys_out=None,
              counts_out=None, d_n_out=None, sync: bool = True, ws=None, stream=None):
    """CGA construction (Section V).  Returns (keys, counts) trimmed to U when
    sync, else (keys, counts, d_n_out) untrimmed with the count on device."""
    assert xyz.is_cuda and xyz.dtype == torch.float32 and xyz.is_contiguous()
    n = xyz.shape[0]
    g = grid_struct(grid)
    cap = n if cap is None else int(cap)
    keys = keys_out if keys_out is not None else _cap_tensor(cap, key_dtype(grid), xyz.device)
    cnt = counts_out if counts_out is not None else (
        _cap_tensor(cap, torch.int32, xyz.device) if counts else None)
    wsb = _ws("build", lib.cga_build_workspace_bytes(ctypes.byref(g), n), ws)
    h = _hostcount()
    rc = lib.cga_build(ctypes.byref(g), _ptr(xyz), n, _ptr(keys), _ptr(cnt), cap, _ptr(d_n_out),
                       ctypes.byref(h) if sync else None, _ptr(wsb), wsb.numel(),
                       tune_struct(tune), _stream(stream))
    _check(rc, "cga_build")
    if sync:
        u = h.value
        return keys[:u], (cnt[:u] if cnt is not None else None)
    return keys, cnt, d_n_out


def cga_encode_keys(xyz: torch.Tensor, grid, ws=None, stream=None) -> torch.Tensor:
    n = xyz.shape[0]
    g = grid_struct(grid)
    keys = _cap_tensor(n, key_dtype(grid), xyz.device)
    wsb = _ws("encode", 256, ws)
    _check(lib.cga_encode_keys(ctypes.byref(g), _ptr(xyz), n, _ptr(keys), _ptr(wsb), wsb.numel(),
                               _stream(stream)), "cga_encode_keys")
    _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_encode_keys")
    return keys[:n]


def cga_sort_keys(keys: torch.Tensor, grid, key_bits: int = 0, tune=None, ws=None, stream=None,
                  out=None) -> torch.Tensor:
    n = keys.shape[0]
    g = grid_struct(grid)
    out = out if out is not None else torch.empty_like(keys)
    wsb = _ws("sort", lib.cga_sort_workspace_bytes(ctypes.byref(g), n), ws)
    _check(lib.cga_sort_keys(ctypes.byref(g), _ptr(keys), n, None, key_bits, _ptr(out), _ptr(wsb),
                             wsb.numel(), tune_struct(tune), _stream(stream)), "cga_sort_keys")
    return out


def cga_to_arrays(keys: torch.Tensor, grid, ws=None, stream=None) -> dict:
    """The paper's X_index, X_pointer, Y_index, Y_pointer, Z_index (LINEAR)."""
    n = keys.shape[0]
    g = grid_struct(grid)
    dev = keys.device
    xi = _cap_tensor(n, torch.int32, dev)
    xp = _cap_tensor(n + 1, torch.int64, dev)
    yi = _cap_tensor(n, torch.int32, dev)
    yp = _cap_tensor(n + 1, torch.int64, dev)
    zi = _cap_tensor(n, torch.int32, dev)
    nx, nxy = _hostcount(), _hostcount()
    wsb = _ws("arrays", lib.cga_to_arrays_workspace_bytes(ctypes.byref(g), n), ws)
    _check(lib.cga_to_arrays(ctypes.byref(g), _ptr(keys), n, None, _ptr(xi), _ptr(xp), _ptr(yi),
                             _ptr(yp), _ptr(zi), None, None, ctypes.byref(nx), ctypes.byref(nxy),
                             _ptr(wsb), wsb.numel(), _stream(stream)), "cga_to_arrays")
    return dict(x_index=xi[:nx.value], x_pointer=xp[:nx.value + 1], y_index=yi[:nxy.value],
                y_pointer=yp[:nxy.value + 1], z_index=zi[:n])


def _arrays_args(arr: dict):
    xi, xp, yi, yp, zi = (arr["x_index"], arr["x_pointer"], arr["y_index"], arr["y_pointer"],
                          arr["z_index"])
    return (_ptr(xi), xi.shape[0], None, _ptr(xp), _ptr(yi), yi.shape[0], None, _ptr(yp),
            _ptr(zi), zi.shape[0])


def cga_arrays_lookup(arr: dict, qvox: torch.Tensor, grid, *, out=None, sync: bool = True,
                      ws=None, stream=None) -> torch.Tensor:
    """Point lookup on the five arrays (Section V-A): int64 position in
    Z_index order, -1 when absent.  qvox: (nq, 3) int32 voxel coordinates."""
    g = grid_struct(grid)
    nq = qvox.shape[0]
    pos = out if out is not None else torch.empty(nq, dtype=torch.int64, device=qvox.device)
    wsb = _ws("arrays_ops", lib.cga_arrays_ops_workspace_bytes(), ws)
    _check(lib.cga_arrays_lookup(ctypes.byref(g), *_arrays_args(arr), _ptr(qvox), nq, _ptr(pos),
                                 _ptr(wsb), wsb.numel(), _stream(stream)), "cga_arrays_lookup")
    if sync:
        _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_arrays_lookup")
    return pos


def cga_arrays_nn(arr: dict, queries: torch.Tensor, grid, *, idx_out=None, d2_out=None,
                  sync: bool = True, ws=None, stream=None):
    """The paper's nearest neighbour on the five arrays (Section V-C):
    (int64 position in Z_index order, uint64 squared distance as int64)."""
    g = grid_struct(grid)
    nq = queries.shape[0]
    dev = queries.device
    idx = idx_out if idx_out is not None else torch.empty(nq, dtype=torch.int64, device=dev)
    d2 = d2_out if d2_out is not None else torch.empty(nq, dtype=torch.int64, device=dev)
    wsb = _ws("arrays_ops", lib.cga_arrays_ops_workspace_bytes(), ws)
    _check(lib.cga_arrays_nn(ctypes.byref(g), *_arrays_args(arr), _ptr(queries), nq, _ptr(idx),
                             _ptr(d2), _ptr(wsb), wsb.numel(), _stream(stream)), "cga_arrays_nn")
    if sync:
        _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_arrays_nn")
    return idx, d2


def cga_temporal_predict(ref_keys: torch.Tensor, ref_values: torch.Tensor, pred_keys: torch.Tensor,
                         pred_values: torch.Tensor, grid, *, window: int = 2, max_iter: int = 20,
                         out: dict = None, sync: bool = True, ws=None, stream=None) -> dict:
    """Temporal prediction (Section V-D): 8-centre k-means of both frames,
    motion vectors, SAD matching in a +-window box, residuals."""
    g = grid_struct(grid)
    nr, npd = ref_keys.shape[0], pred_keys.shape[0]
    dev = pred_keys.device
    o = out if out is not None else dict(
        ref_assign=torch.empty(max(nr, 1), dtype=torch.uint8, device=dev),
        pred_assign=torch.empty(max(npd, 1), dtype=torch.uint8, device=dev),
        centroids=torch.empty((2, 8, 3), dtype=torch.float64, device=dev),
        mv=torch.empty((8, 3), dtype=torch.int32, device=dev),
        iters=torch.empty(2, dtype=torch.int32, device=dev),
        match=torch.empty(max(npd, 1), dtype=torch.int64, device=dev),
        sad=torch.empty(max(npd, 1), dtype=torch.int32, device=dev),
        residual=torch.empty((max(npd, 1), 4), dtype=torch.int16, device=dev))
    wsb = _ws("temporal", lib.cga_temporal_workspace_bytes(), ws)
    _check(lib.cga_temporal_predict(ctypes.byref(g), _ptr(ref_keys), _ptr(ref_values), nr,
                                    _ptr(pred_keys), _ptr(pred_values), npd, int(window),
                                    int(max_iter), _ptr(o["ref_assign"]), _ptr(o["pred_assign"]),
                                    _ptr(o["centroids"]), _ptr(o["mv"]), _ptr(o["iters"]),
                                    _ptr(o["match"]), _ptr(o["sad"]), _ptr(o["residual"]),
                                    _ptr(wsb), wsb.numel(), _stream(stream)),
           "cga_temporal_predict")
    if sync:
        _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_temporal_predict")
        for name, n in (("ref_assign", nr), ("pred_assign", npd), ("match", npd), ("sad", npd),
                        ("residual", npd)):
            o[name] = o[name][:n]
    return o


def cga_merge(a: torch.Tensor, b: torch.Tensor, grid, *, src: bool = False, cap=None, na=None,
              d_na=None, nb=None, d_nb=None, out=None, src_out=None, d_n_out=None,
              sync: bool = True, ws=None, stream=None):
    """Merge, Eq. (1).  Returns (union keys, provenance or None)."""
    na = a.shape[0] if na is None else int(na)
    nb = b.shape[0] if nb is None else int(nb)
    g = grid_struct(grid)
    cap = na + nb if cap is None else int(cap)
    dev = a.device
    out = out if out is not None else _cap_tensor(cap, key_dtype(grid), dev)
    s = src_out if src_out is not None else (_cap_tensor(cap, torch.uint8, dev) if src else None)
    wsb = _ws("merge", lib.cga_merge_workspace_bytes(ctypes.byref(g), na, nb), ws)
    h = _hostcount()
    rc = lib.cga_merge(ctypes.byref(g), _ptr(a), na, _ptr(d_na), _ptr(b), nb, _ptr(d_nb), _ptr(out),
                       _ptr(s), cap, _ptr(d_n_out), ctypes.byref(h) if sync else None, _ptr(wsb),
                       wsb.numel(), _stream(stream))
    _check(rc, "cga_merge")
    if sync:
        u = h.value
        return out[:u], (s[:u] if s is not None else None)
    return out, s, d_n_out


def cga_merge_noalloc(a: torch.Tensor, b: torch.Tensor, grid, *, src: bool = False, cap=None,
                      na=None, d_na=None, nb=None, d_nb=None, out=None, src_out=None,
                      d_n_out=None, sync: bool = True, stream=None):
    """cga_merge over the library's static scratch array (no workspace, no
    allocation inside the call; na + nb <= MERGE_NOALLOC_MAX_KEYS).  Returns
    what cga_merge returns; the output tensors are allocated here unless given."""
    na = a.shape[0] if na is None else int(na)
    nb = b.shape[0] if nb is None else int(nb)
    g = grid_struct(grid)
    cap = na + nb if cap is None else int(cap)
    dev = a.device
    out = out if out is not None else _cap_tensor(cap, key_dtype(grid), dev)
    s = src_out if src_out is not None else (_cap_tensor(cap, torch.uint8, dev) if src else None)
    h = _hostcount()
    rc = lib.cga_merge_noalloc(ctypes.byref(g), _ptr(a), na, _ptr(d_na), _ptr(b), nb, _ptr(d_nb),
                               _ptr(out), _ptr(s), cap, _ptr(d_n_out),
                               ctypes.byref(h) if sync else None, _stream(stream))
    _check(rc, "cga_merge_noalloc")
    if sync:
        u = h.value
        return out[:u], (s[:u] if s is not None else None)
    return out, s, d_n_out


def cga_project(keys: torch.Tensor, grid, drop_axis: int, *, counts: bool = True, cap=None, n=None,
                d_n=None, out=None, counts_out=None, d_n_out=None, tune=None, sync: bool = True,
                ws=None, stream=None):
    """Orthogonal projection, Eq. (3): (sorted unique 2-D keys, voxel counts)."""
    n = keys.shape[0] if n is None else int(n)
    g = grid_struct(grid)
    cap = n if cap is None else int(cap)
    dev = keys.device
    out = out if out is not None else _cap_tensor(cap, key2_dtype(grid), dev)
    cnt = counts_out if counts_out is not None else (
        _cap_tensor(cap, torch.int32, dev) if counts else None)
    wsb = _ws("project", lib.cga_project_workspace_bytes(ctypes.byref(g), n), ws)
    h = _hostcount()
    rc = lib.cga_project(ctypes.byref(g), _ptr(keys), n, _ptr(d_n), int(drop_axis), _ptr(out),
                         _ptr(cnt), cap, _ptr(d_n_out), ctypes.byref(h) if sync else None,
                         _ptr(wsb), wsb.numel(), tune_struct(tune), _stream(stream))
    _check(rc, "cga_project")
    if sync:
        u = h.value
        return out[:u], (cnt[:u] if cnt is not None else None)
    return out, cnt, d_n_out


def cga_knn(keys: torch.Tensor, queries: torch.Tensor, grid, k: int, *, n=None, d_n=None,
            idx_out=None, d2_out=None, sync: bool = True, ws=None, stream=None):
    """k-NN, Eq. (7)-(8): (int64 indices, uint64 squared distances as int64)."""
    n = keys.shape[0] if n is None else int(n)
    nq = queries.shape[0]
    g = grid_struct(grid)
    dev = queries.device
    idx = idx_out if idx_out is not None else torch.empty((nq, k), dtype=torch.int64, device=dev)
    d2 = d2_out if d2_out is not None else torch.empty((nq, k), dtype=torch.int64, device=dev)
    wsb = _ws("knn", lib.cga_knn_workspace_bytes(ctypes.byref(g), n, nq), ws)
    rc = lib.cga_knn(ctypes.byref(g), _ptr(keys), n, _ptr(d_n), _ptr(queries), nq, int(k),
                     _ptr(idx), _ptr(d2), _ptr(wsb), wsb.numel(), _stream(stream))
    _check(rc, "cga_knn")
    if sync:
        _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_knn")
    return idx, d2


def cga_knn_count(keys: torch.Tensor, queries: torch.Tensor, grid, k: int, *, n=None, d_n=None,
                  idx_out=None, d2_out=None, ws=None, stream=None):
    """cga_knn built with work counters: (indices, squared distances, work)
    where work = {node_loads, dense_loads, voxels_offered, steps}, totals
    over all queries (synchronises)."""
    n = keys.shape[0] if n is None else int(n)
    nq = queries.shape[0]
    g = grid_struct(grid)
    dev = queries.device
    idx = idx_out if idx_out is not None else torch.empty((nq, k), dtype=torch.int64, device=dev)
    d2 = d2_out if d2_out is not None else torch.empty((nq, k), dtype=torch.int64, device=dev)
    work = torch.zeros(4, dtype=torch.int64, device=dev)
    wsb = _ws("knn", lib.cga_knn_workspace_bytes(ctypes.byref(g), n, nq), ws)
    rc = lib.cga_knn_count(ctypes.byref(g), _ptr(keys), n, _ptr(d_n), _ptr(queries), nq, int(k),
                           _ptr(idx), _ptr(d2), _ptr(work), _ptr(wsb), wsb.numel(), _stream(stream))
    _check(rc, "cga_knn_count")
    _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_knn_count")
    w = [int(x) for x in work.cpu().tolist()]
    return idx, d2, dict(zip(("node_loads", "dense_loads", "voxels_offered", "steps"), w))


VALUES_BASE, VALUES_AVERAGE = 0, 1


def cga_voxel_values(xyz: torch.Tensor, attr: torch.Tensor, keys: torch.Tensor, grid, *, u=None,
                     d_u=None, out=None, sync: bool = True, ws=None, stream=None) -> torch.Tensor:
    """Value array (Section V): per-voxel channel averages of the points'
    packed 4 x 8-bit attributes (int32 tensor of uint32 bit patterns)."""
    n = xyz.shape[0]
    u = keys.shape[0] if u is None else int(u)
    g = grid_struct(grid)
    vals = out if out is not None else torch.empty(max(u, 1), dtype=torch.int32, device=keys.device)
    wsb = _ws("values", lib.cga_voxel_values_workspace_bytes(ctypes.byref(g), n), ws)
    _check(lib.cga_voxel_values(ctypes.byref(g), _ptr(xyz), n, _ptr(attr), _ptr(keys), u, _ptr(d_u),
                                _ptr(vals), _ptr(wsb), wsb.numel(), _stream(stream)),
           "cga_voxel_values")
    if sync:
        _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_voxel_values")
        return vals[:u]
    return vals


def cga_merge_values(ka, va, kb, vb, km, grid, policy: int, *, na=None, d_na=None, nb=None,
                     d_nb=None, nm=None, d_nm=None, out=None, sync: bool = True, ws=None,
                     stream=None) -> torch.Tensor:
    """Values of the union km of two CGAs (Eq. (1)), base or average on overlap."""
    na = ka.shape[0] if na is None else int(na)
    nb = kb.shape[0] if nb is None else int(nb)
    nm = km.shape[0] if nm is None else int(nm)
    g = grid_struct(grid)
    vals = out if out is not None else torch.empty(max(nm, 1), dtype=torch.int32, device=km.device)
    wsb = _ws("merge_values", lib.cga_merge_values_workspace_bytes(), ws)
    _check(lib.cga_merge_values(ctypes.byref(g), _ptr(ka), _ptr(va), na, _ptr(d_na), _ptr(kb),
                                _ptr(vb), nb, _ptr(d_nb), _ptr(km), nm, _ptr(d_nm), int(policy),
                                _ptr(vals), _ptr(wsb), wsb.numel(), _stream(stream)),
           "cga_merge_values")
    if sync:
        _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_merge_values")
        return vals[:nm]
    return vals


def occupancy_bound(n: int, depth: int) -> int:
    """Most occupancy codes n voxels can have: min(n, 8^(depth - L)) per level."""
    return max(1, sum(min(n, 8 ** (depth - L)) for L in range(1, depth + 1)))


def cga_occupancy(keys: torch.Tensor, grid, *, n=None, d_n=None, occ_out=None, counts_out=None,
                  sync: bool = True, ws=None, stream=None):
    """Octree occupancy codes (Section II-E), root first, level by level:
    (uint8 codes, int64 cells per level).  Trimmed to the code count when sync."""
    n = keys.shape[0] if n is None else int(n)
    g = grid_struct(grid)
    dev = keys.device
    occ = occ_out if occ_out is not None else torch.empty(occupancy_bound(n, grid.depth),
                                                          dtype=torch.uint8, device=dev)
    counts = counts_out if counts_out is not None else torch.empty(grid.depth + 1,
                                                                   dtype=torch.int64, device=dev)
    wsb = _ws("occupancy", lib.cga_occupancy_workspace_bytes(ctypes.byref(g), n), ws)
    _check(lib.cga_occupancy(ctypes.byref(g), _ptr(keys), n, _ptr(d_n), _ptr(occ), occ.numel(),
                             _ptr(counts), _ptr(wsb), wsb.numel(), _stream(stream)), "cga_occupancy")
    if sync:
        _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_occupancy")
        total = int(counts[1:].sum().item())
        return occ[:total], counts
    return occ, counts


def cga_binary_lookup(keys: torch.Tensor, q: torch.Tensor, *, n=None, d_n=None, rank_out=None,
                      found_out=None, stream=None):
    """Lower bound + membership by plain binary search."""
    n = keys.shape[0] if n is None else int(n)
    nq = q.shape[0]
    rank = rank_out if rank_out is not None else torch.empty(nq, dtype=torch.int64, device=q.device)
    found = found_out if found_out is not None else torch.empty(nq, dtype=torch.uint8,
                                                                device=q.device)
    _check(lib.cga_binary_lookup(_ptr(keys), n, _ptr(d_n), _ptr(q), nq, _ptr(rank), _ptr(found),
                                 _stream(stream)), "cga_binary_lookup")
    return rank, found


# ----------------------------------------------------------- learned index
LEAF_LINEAR = 0
LEAF_MLP = 1


def index_params(n_leaves=4096, leaf_kind=LEAF_MLP, epochs=50, lr=1e-4,
                 root_segments=1024) -> cga_index_params:
    p = cga_index_params()
    p.n_leaves, p.leaf_kind, p.epochs, p.lr = int(n_leaves), int(leaf_kind), int(epochs), float(lr)
    p.root_segments = int(root_segments)
    return p


def cga_index_train(keys: torch.Tensor, n=None, *, n_leaves=4096, leaf_kind=LEAF_MLP, epochs=50,
                    lr=1e-4, root_segments=1024, out=None, ws=None, stream=None) -> torch.Tensor:
    """Train the learned index of a sorted unique uint64 key array (int64
    tensor of bit patterns).  Returns the index buffer (uint8 tensor)."""
    n = keys.shape[0] if n is None else int(n)
    p = index_params(n_leaves, leaf_kind, epochs, lr, root_segments)
    nb = lib.cga_index_bytes(ctypes.byref(p))
    if nb == 0:
        raise CgaError(EINVAL, "cga_index_train")
    idx = out if out is not None else torch.empty(nb, dtype=torch.uint8, device=keys.device)
    wsb = _ws("index_train", lib.cga_index_train_workspace_bytes(ctypes.byref(p), n), ws)
    _check(lib.cga_index_train(_ptr(keys), n, ctypes.byref(p), _ptr(idx), idx.numel(), _ptr(wsb),
                               wsb.numel(), _stream(stream)), "cga_index_train")
    return idx


def cga_index_lookup(index: torch.Tensor, keys: torch.Tensor, q: torch.Tensor, *, n=None,
                     rank_out=None, found_out=None, fallbacks_out=None, sync: bool = True,
                     ws=None, stream=None):
    """Learned lookup: (rank int64, found uint8, fallbacks) -- fallbacks is an
    int when sync, else the device counter tensor."""
    n = keys.shape[0] if n is None else int(n)
    nq = q.shape[0]
    dev = q.device
    rank = rank_out if rank_out is not None else torch.empty(nq, dtype=torch.int64, device=dev)
    found = found_out if found_out is not None else torch.empty(nq, dtype=torch.uint8, device=dev)
    fb = fallbacks_out if fallbacks_out is not None else torch.zeros(1, dtype=torch.int64, device=dev)
    wsb = _ws("index_lookup", lib.cga_index_lookup_workspace_bytes(), ws)
    _check(lib.cga_index_lookup(_ptr(index), _ptr(keys), n, _ptr(q), nq, _ptr(rank), _ptr(found),
                                _ptr(fb), _ptr(wsb), wsb.numel(), _stream(stream)),
           "cga_index_lookup")
    if sync:
        _check(lib.cga_ws_status(_ptr(wsb), _stream(stream)), "cga_index_lookup")
        return rank, found, int(fb.item())
    return rank, found, fb


def cga_index_stats(index: torch.Tensor, n_leaves: int, stream=None):
    """Per-leaf (window width, key count) of a trained index."""
    w = torch.empty(n_leaves, dtype=torch.int32, device=index.device)
    c = torch.empty(n_leaves, dtype=torch.int64, device=index.device)
    _check(lib.cga_index_stats(_ptr(index), _ptr(w), _ptr(c), _stream(stream)), "cga_index_stats")
    return w, c


def cga_mlp_loss_grad(params: torch.Tensor, x: torch.Tensor, t: torch.Tensor, stream=None):
    """(loss, gradient[49]) of one leaf network, as the training computes them."""
    g = torch.empty(49, dtype=torch.float64, device=params.device)
    loss = torch.empty(1, dtype=torch.float64, device=params.device)
    _check(lib.cga_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss),
                                 _stream(stream)), "cga_mlp_loss_grad")
    return float(loss.item()), g


# ---------------------------------------------------------------- batched
class BatchOutputs:
    """Device outputs of one batched build + pair merge."""

    def __init__(self, grid, nframes: int, n: int, device="cuda", counts=True):
        kt = key_dtype(grid)
        self.keys = _cap_tensor(n, kt, device)
        self.counts = _cap_tensor(n, torch.int32, device) if counts else None
        self.key_off = torch.zeros(nframes + 1, dtype=torch.int64, device=device)
        self.merged = _cap_tensor(2 * n, kt, device)
        self.merged_off = _cap_tensor(max(nframes - 1, 1), torch.int64, device)
        self.merged_cnt = _cap_tensor(max(nframes - 1, 1), torch.int64, device)

    def frame(self, f: int):
        o = self.key_off.cpu().tolist()
        return self.keys[o[f]:o[f + 1]]

    def pair(self, f: int):
        s0, c = int(self.merged_off[f].item()), int(self.merged_cnt[f].item())
        return self.merged[s0:s0 + c]


def _batch_args(grid, xyz, off, out, tune, wsb):
    g = grid_struct(grid)
    nf = off.shape[0] - 1
    return (ctypes.byref(g), _ptr(xyz), _ptr(off), nf, xyz.shape[0], _ptr(out.keys), _ptr(out.counts),
            _ptr(out.key_off), _ptr(out.merged), _ptr(out.merged_off), _ptr(out.merged_cnt),
            tune_struct(tune), _ptr(wsb), wsb.numel()), g


def cga_batch_sort_bits(grid, nframes: int) -> int:
    """Key bits the batched sort's passes cover (the autotuner's key_bits)."""
    g = grid_struct(grid)
    return int(lib.cga_batch_sort_bits(ctypes.byref(g), nframes))


def cga_batch_build_merge(xyz: torch.Tensor, off: torch.Tensor, grid, *, out=None, tune=None,
                          ws=None, stream=None) -> BatchOutputs:
    """Build every frame's CGA and merge each consecutive pair (device sizes)."""
    nf = off.shape[0] - 1
    out = out if out is not None else BatchOutputs(grid, nf, xyz.shape[0], xyz.device)
    g = grid_struct(grid)
    wsb = _ws("batch", lib.cga_batch_workspace_bytes(ctypes.byref(g), nf, xyz.shape[0]), ws)
    args, _ = _batch_args(grid, xyz, off, out, tune, wsb)
    _check(lib.cga_batch_build_merge(*args, _stream(stream)), "cga_batch_build_merge")
    return out


class BatchGraph:
    """The batched build + pair merge captured once as an executable graph over
    fixed buffers; launch() replays it on a stream."""

    def __init__(self, xyz, off, grid, out=None, tune=None, ws=None):
        nf = off.shape[0] - 1
        self.out = out if out is not None else BatchOutputs(grid, nf, xyz.shape[0], xyz.device)
        g = grid_struct(grid)
        self.wsb = _ws("batch_graph", lib.cga_batch_workspace_bytes(ctypes.byref(g), nf,
                                                                    xyz.shape[0]), ws)
        self._keep = (xyz, off)
        args, self._g = _batch_args(grid, xyz, off, self.out, tune, self.wsb)
        h = ctypes.c_void_p()
        _check(lib.cga_batch_graph_create(*args, ctypes.byref(h)), "cga_batch_graph_create")
        self.handle = h

    def launch(self, stream=None):
        _check(lib.cga_batch_graph_launch(self.handle, _stream(stream)), "cga_batch_graph_launch")

    def status(self, stream=None):
        return lib.cga_ws_status(_ptr(self.wsb), _stream(stream))

    def close(self):
        if self.handle:
            lib.cga_batch_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cga_autotune_sort(keys=None, key_bytes=8, key_bits=64, n=None, ws=None, stream=None):
    """Time every compiled (radix bits, tile items) on these keys (or synthetic
    ones) and record the fastest; returns (radix_bits, tile_items, ms)."""
    if keys is not None:
        n = keys.shape[0] if n is None else int(n)
        key_bytes = keys.element_size()
    wsb = _ws("autotune", lib.cga_autotune_workspace_bytes(key_bytes, n), ws)
    best = cga_tune()
    ms = ctypes.c_float()
    _check(lib.cga_autotune_sort(_ptr(keys), key_bytes, key_bits, n, _ptr(wsb), wsb.numel(),
                                 ctypes.byref(best), ctypes.byref(ms), _stream(stream)),
           "cga_autotune_sort")
    return best.radix_bits, best.tile_items, ms.value


# ------------------------------------------------------------------ timing
def cga_prof_enable(labels=None):
    """Bracket launches of the given kernel labels (None = all) with events."""
    f = ",".join(labels) if labels else None
    _check(lib.cga_prof_enable(f.encode() if f else None), "cga_prof_enable")


def cga_prof_disable():
    lib.cga_prof_disable()


def cga_prof_reset():
    _check(lib.cga_prof_reset(), "cga_prof_reset")


def cga_stream_probe(src: torch.Tensor, dst, nbytes: int, mode: int, blocks: int, stream=None):
    """Enqueue one bandwidth-probe launch (0 = copy src -> dst, 1 = read src)."""
    _check(lib.cga_stream_probe(_ptr(src), _ptr(dst), int(nbytes), int(mode), int(blocks),
                                _stream(stream)), "cga_stream_probe")


def cga_prof_read(label: str):
    """(total milliseconds, launches) of one kernel label since the reset."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib.cga_prof_read(label.encode(), ctypes.byref(ms), ctypes.byref(n)), "cga_prof_read")
    return ms.value, n.value
