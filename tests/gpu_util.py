"""Helpers for the GPU parity tests: move library outputs to numpy."""
import numpy as np
import torch


def off_np(t):
    return t.cpu().numpy().astype(np.uint64)


def nodes_np(t):
    return t.cpu().numpy().view(np.uint32)


def to_dev_u64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def to_dev_u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if a.size == 0:
        return torch.zeros(1, dtype=torch.int32, device="cuda")[:0]
    return torch.from_numpy(a.view(np.int32)).cuda()


def say(*args):
    print(*args, flush=True)
