"""Helpers for the GPU tests: device handles and tolerances."""
import numpy as np


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm((a - b).reshape(-1))
    n = np.linalg.norm(b.reshape(-1))
    return d / n if n > 0 else d


def subspace_dist(F1, F2):
    """||F1 F1^T - F2 F2^T||_2 (basis-free comparison of column spaces)."""
    return float(np.linalg.norm(F1 @ F1.T - F2 @ F2.T, 2))


def to_dev(x, dtype=None):
    torch, dev = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)
