"""Mixed-precision path: split-BF16x3 / FP32 pipeline + FP64 Ogita-Aishima
refinement (evd_dsyevd_mixed).  Gates are the mixed path's own acceptance
(reading A of the 1e-13 scaled residual): ||A X - X L||_F/(n ||A||_F),
||X^T X - I||_F / n and the eigenvalue error vs the oracle / known spectrum."""
import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import workloads as W

pytestmark = pytest.mark.gpu


def run_mixed(A, sweeps, b=0):
    from paper_2511_16174_amd import evd
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    w, Q, stats = evd.eigh_mixed(At, sweeps=sweeps, b=b)
    torch.cuda.synchronize()
    return w.cpu().numpy(), Q.cpu().numpy(), stats.cpu().numpy()


def scaled_res(A, w, Q):
    n = A.shape[0]
    return np.linalg.norm(A @ Q - Q * w[None, :]) / (n * np.linalg.norm(A))


def scaled_orth(Q):
    n = Q.shape[0]
    return np.linalg.norm(Q.T @ Q - np.eye(n)) / n


def test_mixed_unrefined_is_bf16x3_accurate():
    A = W.gaussian_sym(512, seed=1)
    w, Q, st = run_mixed(A, sweeps=0, b=32)
    r = scaled_res(A, w, Q)
    assert 1e-12 < r < 1e-5          # far from FP64, within the split's ~17 bits
    assert abs(st[4] - r) <= 1e-3 * r + 1e-18  # the reported residual is the real one


@pytest.mark.parametrize("n,seed", [(256, 2), (1024, 3)])
def test_mixed_refined_gaussian(n, seed):
    A = W.gaussian_sym(n, seed=seed, scaled=True)
    w_ref = oracle.syev(A, jobz="N")
    res = []
    for sw in (0, 1, 2, 3):
        w, Q, st = run_mixed(A, sweeps=sw, b=32)
        res.append(scaled_res(A, w, Q))
    assert res[2] <= res[0]
    w, Q, st = run_mixed(A, sweeps=3, b=32)
    assert scaled_res(A, w, Q) <= 1e-13
    assert scaled_orth(Q) <= 1e-13
    assert M.eig_error(w, w_ref) <= 1e-12
    assert np.all(np.diff(w) >= 0)


def test_mixed_known_spectrum_well_separated():
    n = 600
    A, lam = W.known_spectrum(n, seed=5, spectrum="uniform", reflectors=16)
    w, Q, st = run_mixed(A, sweeps=3, b=32)
    assert M.eig_error(w, lam) <= 1e-12
    assert scaled_res(A, w, Q) <= 1e-13 and scaled_orth(Q) <= 1e-13


def test_mixed_clustered_spectrum():
    """16 clusters of 8 eigenvalues at relative gaps 1e-8: the clusters are
    resolved by the Rayleigh-Ritz step of the refinement."""
    n = 512
    A, lam = W.known_spectrum(n, seed=8, spectrum="clustered", reflectors=16)
    w, Q, st = run_mixed(A, sweeps=3, b=32)
    print(f"clustered n={n}: eta={M.eig_error(w, lam):.2e} res={scaled_res(A, w, Q):.2e} "
          f"orth={scaled_orth(Q):.2e} clusters={st[5]:.0f} kmax={st[6]:.0f}")
    assert M.eig_error(w, lam) <= 1e-12
    assert scaled_res(A, w, Q) <= 1e-13 and scaled_orth(Q) <= 1e-13


def test_mixed_logspaced_report():
    """Log-spaced |lambda| over [1e-6, 1] with random signs (dense clusters
    near 0): the refinement must not make things worse; the achieved
    accuracy is recorded."""
    n = 1024
    A, lam = W.known_spectrum(n, seed=6, spectrum="logspaced", reflectors=16)
    w0, Q0, _ = run_mixed(A, sweeps=0, b=32)
    w2, Q2, st = run_mixed(A, sweeps=3, b=32)
    r0, r2 = scaled_res(A, w0, Q0), scaled_res(A, w2, Q2)
    print(f"logspaced n={n}: res0={r0:.2e} res3={r2:.2e} eta={M.eig_error(w2, lam):.2e} "
          f"orth={scaled_orth(Q2):.2e} delta={st[0]:.2e}")
    print(f"  clusters={st[5]:.0f} kmax={st[6]:.0f}")
    assert r2 <= r0
    assert M.eig_error(w2, lam) <= 1e-12
