"""Stage 2 (bulge chasing) on the GPU: the tridiagonal T it returns has the
band's spectrum (exact Sturm counts at oracle midpoints), the stored
reflectors reproduce T = Q_b^T B Q_b, and the result does not depend on the
number of persistent wavefronts (no race)."""
import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import workloads as W
from tests.gpu_helpers import band_to_dense, from_dev, to_dev, work_dev, zeros_dev

pytestmark = pytest.mark.gpu


def random_band(n, b, seed):
    r = W.rng(seed)
    A = r.standard_normal((n, n))
    A = 0.5 * (A + A.T)
    for i in range(n):
        for j in range(n):
            if abs(i - j) > b:
                A[i, j] = 0.0
    return A


def band_storage(B, b):
    n = B.shape[0]
    ldab = 2 * b + 1
    AB = np.zeros((ldab, n))
    for d in range(b + 1):
        for j in range(n - d):
            AB[d, j] = B[j + d, j]
    return AB


def run_bc(B, b, jobz="V", waves=0):
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    ctx.set_param("bc_waves", waves)
    n = B.shape[0]
    ldab = 2 * b + 1
    dAB = to_dev(band_storage(B, b))
    dd, de = zeros_dev(n), zeros_dev(max(n - 1, 1))
    steps = evd.evd_bc_num_steps(n, b)
    dV = zeros_dev(max(steps * n * b, 1))
    dT = zeros_dev(max(steps * n, 1))
    wb = ctx.evd_dsb2st_work_size(n)
    work = work_dev(wb)
    ctx.evd_dsb2st(jobz, n, b, dAB, ldab, dd, de, dV, dT, work, wb)
    torch.cuda.synchronize()
    ctx.set_param("bc_waves", 0)
    d = dd.cpu().numpy()[:n]
    e = de.cpu().numpy()[: max(n - 1, 0)]
    V = dV.cpu().numpy()[: steps * n * b].reshape(steps, n, b)
    TAU = dT.cpu().numpy()[: steps * n].reshape(steps, n)
    return d, e, V, TAU, steps


def q_from_reflectors(n, b, V, TAU, steps):
    """Q_b = H_1 H_2 ... in generation order (sweep-major, then step)."""
    Q = np.eye(n)
    for c in range(n - 2):
        for s in range(steps):
            t = TAU[s, c]
            r = c + 1 + s * b
            if r >= n:
                break
            if t == 0.0:
                continue
            m = min(b, n - r)
            v = V[s, c, :m]
            X = Q[:, r:r + m]
            Q[:, r:r + m] = X - t * np.outer(X @ v, v)
    return Q


@pytest.mark.parametrize("n,b", [(3, 1), (5, 2), (40, 4), (100, 8), (257, 16), (300, 32), (200, 64), (130, 64)])
def test_bc_spectrum_and_reflectors(n, b):
    B = random_band(n, b, seed=n * 3 + b)
    d, e, V, TAU, steps = run_bc(B, b)
    w_ref = oracle.syev(B, jobz="N")
    w_t = oracle.stev(d, e, jobz="N")
    assert M.eig_error(w_t, w_ref) <= 1e-13
    # exact Sturm counts at midpoints of well-separated oracle eigenvalues
    scale = max(abs(w_ref[0]), abs(w_ref[-1]))
    for i in range(n - 1):
        if w_ref[i + 1] - w_ref[i] > 1e-10 * scale:
            assert oracle.sturm(d, e, 0.5 * (w_ref[i] + w_ref[i + 1])) == i + 1
    # the stored reflectors reduce B to T
    Q = q_from_reflectors(n, b, V, TAU, steps)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert M.orthogonality(Q) <= 10
    assert np.linalg.norm(Q.T @ B @ Q - T) / (n * np.linalg.norm(B) * M.EPS) <= 10
    # the first row/column is untouched by all reflectors (Q e_1 = e_1)
    assert d[0] == B[0, 0]


def test_bc_values_only_and_wave_count_do_not_change_result():
    n, b = 500, 16
    B = random_band(n, b, seed=77)
    d0, e0, *_ = run_bc(B, b, "V", waves=0)
    for waves in (1, 3, 17):
        d1, e1, *_ = run_bc(B, b, "V", waves=waves)
        assert np.array_equal(d0, d1) and np.array_equal(e0, e1)
    d2, e2, *_ = run_bc(B, b, "N")
    assert np.array_equal(d0, d2) and np.array_equal(e0, e2)


def test_bc_on_tridiagonal_input_is_identity():
    """A band matrix that is already tridiagonal: every reflector is trivial."""
    n, b = 64, 8
    B = W.laplacian_1d(n)
    d, e, V, TAU, steps = run_bc(B, b)
    assert np.all(TAU == 0.0)
    assert np.array_equal(d, np.diag(B)) and np.array_equal(e, np.diag(B, -1))
