"""Stage 1 (SBR, Eq. 1) on the GPU: band eigenvalues vs the oracle, and the
returned panel reflectors reproduce A = Q_s B Q_s^T."""
import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import workloads as W
from tests.gpu_helpers import band_to_dense, from_dev, to_dev, work_dev, zeros_dev

pytestmark = pytest.mark.gpu


def run_sbr(A, b, uplo="L"):
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    n = A.shape[0]
    ldab = 2 * b + 1
    dA = to_dev(A)
    dAB = zeros_dev(ldab * n)
    p = evd.evd_sbr_num_panels(n, b)
    dT = zeros_dev(max(p, 1) * b * b)
    wb = ctx.evd_dsy2sb_work_size(n, b)
    work = work_dev(wb)
    ctx.evd_dsy2sb(uplo, n, b, dA, n, dAB, ldab, dT, work, wb)
    torch.cuda.synchronize()
    AB = from_dev(dAB, ldab, n)
    Aout = from_dev(dA, n, n)
    T = dT.cpu().numpy()[: p * b * b].reshape(p, b, b).transpose(0, 2, 1) if p else np.zeros((0, b, b))
    return AB, Aout, T, p


def q_from_panels(Aout, T, n, b, p):
    Q = np.eye(n)
    for k in range(p):
        i0 = (k + 1) * b
        Y = Aout[i0:, k * b:(k + 1) * b]
        H = np.eye(n)
        H[i0:, i0:] -= Y @ T[k] @ Y.T
        Q = Q @ H
    return Q


@pytest.mark.parametrize("n,b", [(3, 1), (10, 4), (66, 64), (67, 64), (100, 8), (256, 16), (333, 32),
                                 (512, 32), (300, 64), (130, 2)])
def test_sbr_band_and_reflectors(n, b):
    A = W.gaussian_sym(n, seed=n + b)
    AB, Aout, T, p = run_sbr(A, b)
    ldab = 2 * b + 1
    assert np.all(AB[b + 1:, :] == 0.0)
    B = band_to_dense(AB, n, b, ldab)
    w_ref = oracle.syev(A, jobz="N")
    assert M.eig_error(np.linalg.eigvalsh(B), w_ref) <= 1e-13
    # T_k upper triangular, Y_k unit lower trapezoidal
    for k in range(p):
        assert np.all(np.tril(T[k], -1) == 0.0)
        i0 = (k + 1) * b
        Y = Aout[i0:, k * b:(k + 1) * b]
        r = min(Y.shape[0], b)
        assert np.all(np.triu(Y[:r], 1) == 0.0) and np.all(np.diag(Y[:r]) == 1.0)
    Q = q_from_panels(Aout, T, n, b, p)
    assert M.orthogonality(Q) <= 10
    rec = np.linalg.norm(Q @ B @ Q.T - A) / (n * np.linalg.norm(A) * M.EPS)
    assert rec <= 10


def test_sbr_upper_matches_lower():
    n, b = 200, 16
    A = W.gaussian_sym(n, seed=4)
    AB_l, _, _, _ = run_sbr(A, b, "L")
    junk = np.triu(A) + np.tril(np.full_like(A, 7e7), -1)  # lower triangle garbage
    AB_u, _, _, _ = run_sbr(junk, b, "U")
    assert np.array_equal(AB_l, AB_u)


def test_sbr_known_spectrum():
    n, b = 400, 32
    A, lam = W.known_spectrum(n, seed=2, spectrum="clustered", reflectors=16)
    AB, _, _, _ = run_sbr(A, b)
    B = band_to_dense(AB, n, b, 2 * b + 1)
    assert M.eig_error(np.linalg.eigvalsh(B), lam) <= 1e-13


@pytest.mark.parametrize("n,b", [(700, 32), (530, 64)])
def test_sbr_double_blocking_matches_single(n, b):
    """The deferred (double-blocked) update and one update per panel give the
    same band up to rounding, and both reconstruct A."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    A = W.gaussian_sym(n, seed=11)
    try:
        ctx.set_param("sbr_nb", b)
        AB1, Aout1, T1, p = run_sbr(A, b)
    finally:
        ctx.set_param("sbr_nb", 0)
    AB2, Aout2, T2, _ = run_sbr(A, b)
    ldab = 2 * b + 1
    B1 = band_to_dense(AB1, n, b, ldab)
    B2 = band_to_dense(AB2, n, b, ldab)
    assert np.abs(B1 - B2).max() <= 1e-11 * np.abs(A).max() * n
    for Aout, T, B in ((Aout1, T1, B1), (Aout2, T2, B2)):
        Q = q_from_panels(Aout, T, n, b, p)
        rec = np.linalg.norm(Q @ B @ Q.T - A) / (n * np.linalg.norm(A) * M.EPS)
        assert rec <= 10


@pytest.mark.parametrize("n,b,wgs", [(1100, 64, 0), (800, 32, 0), (1100, 64, 16), (1100, 32, 16), (1100, 16, 16),
                                     (300, 4, 8), (200, 1, 4)])
def test_sbr_panel_row_slices(n, b, wgs):
    """Panel workgroups holding the most rows their registers take (the
    default, 512 rows at b = 64: the longest per-column work, as at the
    largest n) or the rows spread over several workgroups ("panel_wgs"),
    also for narrow panels whose columns span several wavefronts (b <= 4).
    The band and reflectors must reconstruct A, and two runs must agree bit
    for bit (every workgroup sums the partial-sum records in one fixed
    order)."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    A = W.gaussian_sym(n, seed=n + wgs)
    try:
        ctx.set_param("panel_wgs", wgs)
        AB1, Aout, T, p = run_sbr(A, b)
        AB2, _, _, _ = run_sbr(A, b)
    finally:
        ctx.set_param("panel_wgs", 0)
    assert np.array_equal(AB1, AB2)
    B = band_to_dense(AB1, n, b, 2 * b + 1)
    Q = q_from_panels(Aout, T, n, b, p)
    assert M.orthogonality(Q) <= 10
    rec = np.linalg.norm(Q @ B @ Q.T - A) / (n * np.linalg.norm(A) * M.EPS)
    assert rec <= 10


@pytest.mark.parametrize("n,wgs", [(66, 0), (67, 0), (130, 0), (300, 0), (1100, 0), (1100, 16), (2500, 0)])
def test_sbr_panel_column_layout_matches_generic(n, wgs):
    """b = 64 panels in the column layout (default: each wavefront holds eight
    whole columns) and in the generic layout ("panel_generic" = 1) give the
    same band up to the order of the sums, both reconstruct A, and the
    column layout is reproducible bit for bit; panels shorter than b (n = 67),
    partial last workgroups and rows spread over 15 workgroups included."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    b = 64
    A = W.gaussian_sym(n, seed=3 * n + wgs)
    try:
        ctx.set_param("panel_wgs", wgs)
        AB1, Aout1, T1, p = run_sbr(A, b)
        AB1b, _, _, _ = run_sbr(A, b)
        ctx.set_param("panel_generic", 1)
        AB2, Aout2, T2, _ = run_sbr(A, b)
    finally:
        ctx.set_param("panel_wgs", 0)
        ctx.set_param("panel_generic", 0)
    assert np.array_equal(AB1, AB1b)
    ldab = 2 * b + 1
    B1 = band_to_dense(AB1, n, b, ldab)
    B2 = band_to_dense(AB2, n, b, ldab)
    assert np.abs(B1 - B2).max() <= 1e-11 * np.abs(A).max() * n
    for Aout, T, B in ((Aout1, T1, B1), (Aout2, T2, B2)):
        Q = q_from_panels(Aout, T, n, b, p)
        assert M.orthogonality(Q) <= 10
        rec = np.linalg.norm(Q @ B @ Q.T - A) / (n * np.linalg.norm(A) * M.EPS)
        assert rec <= 10
