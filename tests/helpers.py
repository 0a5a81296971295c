"""Shared test helpers: device transfer and unsigned views."""
import numpy as np
import torch


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def u64(t):
    """GPU key tensor (int32 / int64 bit patterns) -> numpy uint64."""
    a = t.detach().cpu().numpy()
    if a.dtype == np.int32:
        return a.view(np.uint32).astype(np.uint64)
    return a.view(np.uint64)


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def keys_dev(keys_u64, grid):
    """numpy uint64 keys -> device tensor of the grid's key width."""
    if 3 * grid.depth > 32:
        return dev(keys_u64.astype(np.uint64).view(np.int64))
    return dev(keys_u64.astype(np.uint32).view(np.int32))


def say(*a):
    print(*a, flush=True)
