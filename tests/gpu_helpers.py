"""Helpers shared by the GPU tests: column-major device buffers via torch."""
import numpy as np


def torch():
    import torch as t
    return t


def to_dev(x):
    """Column-major device copy of a 2-D numpy array (memory = x in Fortran order)."""
    t = torch()
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        return t.from_numpy(x.copy()).cuda()
    return t.from_numpy(np.ascontiguousarray(x.T)).cuda()


def from_dev(t, m, n):
    """Inverse of to_dev for an m x n column-major buffer (leading dimension m)."""
    a = t.detach().cpu().numpy()
    return np.asfortranarray(a.reshape(-1)[: m * n].reshape(n, m).T)


def zeros_dev(count):
    t = torch()
    return t.zeros(max(int(count), 1), dtype=t.float64, device="cuda")


def work_dev(nbytes):
    t = torch()
    return t.empty(max(int(nbytes) // 8 + 32, 32), dtype=t.float64, device="cuda")


def band_to_dense(AB, n, b, ldab):
    """AB (ldab x n, column-major host array) lower band -> full symmetric n x n."""
    B = np.zeros((n, n))
    for d in range(b + 1):
        for j in range(n - d):
            B[j + d, j] = AB[d, j]
            B[j, j + d] = AB[d, j]
    return B
