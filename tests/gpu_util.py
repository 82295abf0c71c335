"""Helpers shared by the GPU parity tests (imported lazily, never by CPU tests)."""
import numpy as np


def lib():
    import paper_1205_4139_amd as fc
    return fc


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def inf_rel(a, b):
    """||a - b||_inf / ||b||_inf."""
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.max(np.abs(a - b))
    s = np.max(np.abs(b))
    return d / s if s > 0 else d


def rand_vec(rng, n, complex_):
    v = rng.standard_normal(n)
    if complex_:
        v = (v + 1j * rng.standard_normal(n)) / np.sqrt(2)
    return v


def omega(rng, N, M):
    return np.sort(rng.choice(N, M, replace=False)).astype(np.int32)
