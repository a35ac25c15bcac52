"""Helpers shared by the GPU tests: host<->device copies of ring arrays."""
import numpy as np
import torch


def dev(a, device="cuda"):
    """numpy uint64/int64 array -> int64 device tensor with the same bits."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a.astype(np.int64, copy=False)).to(device)


def host(ctx, t):
    """device tensor -> numpy uint64 (after both party streams finish)."""
    ctx.sync()
    return t.cpu().numpy().view(np.uint64)


def pair(ctx, p):
    return host(ctx, p.s0), host(ctx, p.s1)


def say(*a):
    print(*a, flush=True)
