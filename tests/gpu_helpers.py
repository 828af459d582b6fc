"""Shared helpers of the GPU parity tests (device transfer and comparisons)."""
import numpy as np


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def announce(*what):
    """Name the case on stdout before the GPU call (kept if a run dies)."""
    print("CASE", *what, flush=True)
