"""cga_merge_noalloc, the merge over the library's static scratch array, for
callers that cannot allocate: called through the C ABI (ctypes) and compared
element by element with cga_merge (caller workspace) and with the oracle's
std::set_union, on two calls in a row, the second with a smaller input, for
both key widths; then a call whose sizes come from device counts below the
host bounds."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from helpers import keys_dev, say, u64

pytestmark = pytest.mark.gpu


def _sets(seed, na, nb, depth):
    """Two sorted unique key sets over 3*depth bits sharing about a third of B."""
    rng = np.random.default_rng(seed)
    top = np.uint64(1) << np.uint64(3 * depth)
    a = np.unique(rng.integers(0, top, na, dtype=np.uint64))
    b = np.unique(np.concatenate([rng.integers(0, top, nb - nb // 3, dtype=np.uint64),
                                  rng.choice(a, nb // 3, replace=False)]))
    return a, b


def _grid(cga, depth):
    return cga.Grid(origin=(0.0, 0.0, 0.0), scale=1.0, depth=depth, key_mode=cga.KEY_MORTON)


def _call_abi(cga, g, a, b, na=None, nb=None, d_na=None, d_nb=None):
    """One cga_merge_noalloc call through ctypes; returns (keys, provenance,
    device count, host count)."""
    na = a.shape[0] if na is None else na
    nb = b.shape[0] if nb is None else nb
    cap = na + nb
    out = torch.full((max(cap, 1),), -1, dtype=cga.key_dtype(g), device="cuda")
    src = torch.zeros(max(cap, 1), dtype=torch.uint8, device="cuda")
    dn = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    h = ctypes.c_int64(-1)
    gs = cga.grid_struct(g)
    ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    rc = cga.lib.cga_merge_noalloc(ctypes.byref(gs), ptr(a), na, ptr(d_na), ptr(b), nb, ptr(d_nb),
                                   ptr(out), ptr(src), cap, ptr(dn), ctypes.byref(h),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == cga.OK, cga.lib.cga_strerror(rc)
    return out, src, int(dn.item()), h.value


@pytest.mark.parametrize("depth", [12, 10])
def test_noalloc_merge_matches_workspace_merge(gpu, depth):
    cga = gpu
    g = _grid(cga, depth)
    for call, (na, nb) in enumerate(((300_000, 250_000), (5_000, 7_001))):
        a_np, b_np = _sets(4100 + 10 * depth + call, na, nb, depth)
        say(f"noalloc merge depth {depth} call {call}: |A|={len(a_np)} |B|={len(b_np)}")
        a, b = keys_dev(a_np, g), keys_dev(b_np, g)
        out, src, dn, h = _call_abi(cga, g, a, b)
        torch.cuda.synchronize()
        want_k, want_s = cga.cga_merge(a, b, g, src=True)
        ref_k, ref_s = oracle.merge(a_np, b_np, depth, g.key_mode)
        assert h == dn == len(ref_k) == want_k.shape[0]
        np.testing.assert_array_equal(u64(out[:h]), u64(want_k))
        np.testing.assert_array_equal(src[:h].cpu().numpy(), want_s.cpu().numpy())
        np.testing.assert_array_equal(u64(out[:h]), ref_k)
        np.testing.assert_array_equal(src[:h].cpu().numpy(), ref_s)
        # nothing written past the union
        assert bool((out[h:] == -1).all())


def test_noalloc_merge_device_counts(gpu):
    """Sizes on the device below the host bounds (a graph-style call)."""
    cga = gpu
    g = _grid(cga, 12)
    a_np, b_np = _sets(4200, 40_000, 30_000, 12)
    a, b = keys_dev(a_np, g), keys_dev(b_np, g)
    ua, ub = len(a_np) - 1234, len(b_np) - 77
    d_na = torch.tensor([ua], dtype=torch.int64, device="cuda")
    d_nb = torch.tensor([ub], dtype=torch.int64, device="cuda")
    out, src, dn, h = _call_abi(cga, g, a, b, d_na=d_na, d_nb=d_nb)
    ref_k, ref_s = oracle.merge(a_np[:ua], b_np[:ub], 12, g.key_mode)
    assert h == dn == len(ref_k)
    np.testing.assert_array_equal(u64(out[:h]), ref_k)
    np.testing.assert_array_equal(src[:h].cpu().numpy(), ref_s)
