"""Stage 3 (tridiagonal divide and conquer, and bisection for eigenvalues
only) on the GPU against closed forms and the oracle's QL."""
import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import workloads as W
from tests.gpu_helpers import from_dev, to_dev, work_dev, zeros_dev

pytestmark = pytest.mark.gpu


def run_dc(d, e, compz="I"):
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    n = d.size
    dd, de = to_dev(d), to_dev(e if n > 1 else np.zeros(1))
    dW = zeros_dev(n)
    dZ = zeros_dev(n * n) if compz == "I" else None
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    wb = ctx.evd_dstedc_work_size(compz, n)
    work = work_dev(wb)
    ctx.evd_dstedc(compz, n, dd, de, dW, dZ, max(n, 1), work, wb, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w = dW.cpu().numpy()[:n]
    Z = from_dev(dZ, n, n) if compz == "I" else None
    return w, Z


def tri(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 100, 513])
def test_dc_laplacian_closed_form(n):
    d, e = 2.0 * np.ones(n), -np.ones(n - 1)
    w, Z = run_dc(d, e)
    lam = W.laplacian_eigenvalues(n)
    assert np.all(np.diff(w) >= 0)
    assert np.max(np.abs(w - lam)) <= 1e-13 * 4
    T = tri(d, e)
    assert M.residual(T, w, Z) <= 10 and M.orthogonality(Z) <= 10
    j = np.arange(1, n + 1)[:, None]
    k = np.arange(1, n + 1)[None, :]
    V = np.sqrt(2.0 / (n + 1)) * np.sin(j * k * np.pi / (n + 1))
    for c in range(n):
        s = np.sign(Z[:, c] @ V[:, c])
        assert np.linalg.norm(Z[:, c] - s * V[:, c]) <= 1e-10


@pytest.mark.parametrize("n,seed", [(5, 1), (200, 2), (1000, 3), (1537, 4)])
def test_dc_random_vs_oracle(n, seed):
    r = W.rng(seed)
    d, e = r.standard_normal(n), r.standard_normal(n - 1)
    w, Z = run_dc(d, e)
    w_ref = oracle.stev(d, e, jobz="N")
    assert M.eig_error(w, w_ref) <= 1e-14 * 8
    T = tri(d, e)
    assert M.residual(T, w, Z) <= 10 and M.orthogonality(Z) <= 10


def test_dc_wilkinson_close_pairs():
    n = 21
    d = np.abs(np.arange(n) - 10.0)
    e = np.ones(n - 1)
    w, Z = run_dc(d, e)
    w_ref = oracle.stev(d, e, jobz="N")
    assert M.eig_error(w, w_ref) <= 1e-14 * 8
    assert M.residual(tri(d, e), w, Z) <= 10 and M.orthogonality(Z) <= 10


@pytest.mark.parametrize("case", ["block_zeros", "constant", "kac", "tiny_offdiag", "glued"])
def test_dc_deflation_heavy(case):
    n = 300
    r = W.rng(9)
    if case == "block_zeros":
        d, e = r.standard_normal(n), r.standard_normal(n - 1)
        e[::7] = 0.0
    elif case == "constant":
        d, e = np.ones(n), np.zeros(n - 1)
        e[n // 2] = 1e-3
    elif case == "kac":
        K = W.kac_matrix(101)
        d, e = np.diag(K).copy(), np.diag(K, -1).copy()
        n = 101
    elif case == "tiny_offdiag":
        d, e = np.sort(r.standard_normal(n)), 1e-12 * r.standard_normal(n - 1)
    else:  # glued Wilkinson matrices
        m = 21
        blk = np.abs(np.arange(m) - 10.0)
        d = np.concatenate([blk] * 10)
        e = np.ones(10 * m - 1)
        e[m - 1::m] = 1e-8
        n = d.size
    w, Z = run_dc(d, e)
    w_ref = oracle.stev(d, e, jobz="N")
    assert M.eig_error(w, w_ref) <= 1e-14 * 8
    assert M.residual(tri(d, e), w, Z) <= 10 and M.orthogonality(Z) <= 10


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (50, 2), (777, 3)])
def test_bisection_values_only(n, seed):
    r = W.rng(seed)
    d, e = r.standard_normal(n), r.standard_normal(max(n - 1, 0))
    w, _ = run_dc(d, e, "N")
    w_ref = oracle.stev(d, e, jobz="N")
    assert np.all(np.diff(w) >= 0)
    assert M.eig_error(w, w_ref) <= 1e-14 * 8


def test_dc_more_merges_than_one_launch_holds():
    """n = 32800 has 16 merge levels; the deepest has 2^15 merges, i.e. 2^16
    merge products, more than one launch's grid can index, so the grouped
    products are issued in parts.  Checked against the closed-form spectrum of
    the 1-D Laplacian and, on sampled columns, A z = lambda z and unit norm
    (the full n x n eigenvector matrix is not copied to the host)."""
    from paper_2511_16174_amd import evd
    import torch
    n = 32800
    ctx = evd.context(0)
    dd = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    de = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    dW = torch.zeros(n, dtype=torch.float64, device="cuda")
    dZ = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    wb = ctx.evd_dstedc_work_size("I", n)
    work = work_dev(wb)
    ctx.evd_dstedc("I", n, dd, de, dW, dZ, n, work, wb, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    w = dW.cpu().numpy()
    lam = W.laplacian_eigenvalues(n)
    assert np.max(np.abs(w - lam)) <= 1e-12 * 4.0
    Zt = dZ.view(n, n)  # row j of Zt = column j of Z
    for j in (0, 1, n // 3, n // 2, n - 2, n - 1):
        z = Zt[j].cpu().numpy()
        Az = 2.0 * z
        Az[1:] -= z[:-1]
        Az[:-1] -= z[1:]
        assert np.linalg.norm(Az - w[j] * z) <= 1e-12 * 4.0 * np.sqrt(n)
        assert abs(np.linalg.norm(z) - 1.0) <= 1e-12 * n


def test_dc_merge_products_direct_lds_match_staged():
    """The top merges at n = 6000 run the grouped products on the kernel whose
    K slices are loaded straight into LDS (a partial last slice zero-filled);
    the eigenpairs are bit for bit those of the register-staged products
    ("gemm_staged" = 1), and match the oracle."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    n = 6000
    rng = np.random.default_rng(6000)
    d, e = rng.standard_normal(n), rng.standard_normal(n - 1)
    out = []
    try:
        for staged in (0, 1):
            ctx.set_param("gemm_staged", staged)
            out.append(run_dc(d, e))
    finally:
        ctx.set_param("gemm_staged", 0)
    (w0, Z0), (w1, Z1) = out
    assert np.array_equal(w0, w1) and np.array_equal(Z0, Z1)
    T = tri(d, e)
    nrm = np.abs(T).sum(axis=1).max()
    assert M.residual(T, w0, Z0) <= 10 and M.orthogonality(Z0) <= 10
    assert np.max(np.abs(np.sort(w0) - np.linalg.eigvalsh(T))) <= 1e-12 * nrm
