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
