"""Helpers shared by the GPU tests: device transfer and tolerances.

The oracle computes every expected value; the library under test is reached
only through its C ABI (paper_1401_5171_amd, ctypes over liboqr.so).
"""
import numpy as np

U = 2.0 ** -53


def to_dev(x):
    import torch
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 2 and x.shape[0] != x.shape[1]:
        # column-major (m, n): upload the transpose contiguously and view it back
        return torch.from_numpy(np.ascontiguousarray(x.T)).cuda().t()
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def to_dev_colmajor(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64).T)).cuda().t()


def to_host(t):
    return t.detach().cpu().numpy()


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
