"""Helpers for the GPU parity tests (inputs from the seeded generators, oracle
on the CPU, library through its C ABI)."""
import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test needs a HIP device")
    return torch


def dev_matrix(A, ld=None):
    from paper_2104_01253_amd import binding
    return binding.colmajor_from_numpy(np.asarray(A, dtype=np.float64), ld=ld)


def dev_vector(x):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relnorm(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def colerr(X, Xref):
    """max_ij |X_ij - Xref_ij| / ||Xref[:, j]||_2: every element against the scale of its
    own reference column (a zero reference column is compared absolutely)."""
    X = np.asarray(X, dtype=np.float64)
    Xref = np.asarray(Xref, dtype=np.float64)
    if Xref.ndim == 1:                       # a vector is one column
        X, Xref = X.reshape(-1, 1), Xref.reshape(-1, 1)
    scale = np.linalg.norm(Xref, axis=0)
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(X - Xref) / scale[None, :])) if X.size else 0.0


def maxerr(x, ref, scale):
    """max_i |x_i - ref_i| / scale."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if x.size == 0:
        return 0.0
    return float(np.max(np.abs(x - ref))) / max(float(scale), 1e-300)
