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


class params:
    """Set context parameters for a block and restore the previous values."""

    def __init__(self, ctx, **kv):
        self.ctx, self.kv, self.saved = ctx, kv, {}

    def __enter__(self):
        for k, v in self.kv.items():
            self.saved[k] = self.ctx.get_param(k)
            self.ctx.set_param(k, v)
        return self.ctx

    def __exit__(self, *exc):
        for k, v in self.saved.items():
            self.ctx.set_param(k, v)
        return False


def device_ratios(A0, w, X, eps=2.0 ** -52):
    """rho_res, rho_orth of the eigenpairs (w, X) of the symmetric A0 (torch
    FP64 tensors on the GPU, X[:, j] the j-th vector), with torch's own FP64
    products (independent of the library under test)."""
    t = torch()
    n = A0.shape[0]
    with t.no_grad():
        R = A0 @ X - X * w[None, :]
        res = (t.linalg.norm(R) / (n * t.linalg.norm(A0) * eps)).item()
        del R
        O = X.t() @ X
        O.diagonal().sub_(1.0)
        orth = (t.linalg.norm(O) / (n * eps)).item()
    return res, orth
