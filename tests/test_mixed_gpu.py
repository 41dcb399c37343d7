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

TARGET = 1e-13


def run_mixed(A, sweeps, b=0, target=0.0, check=True):
    from paper_2511_16174_amd import evd
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    w, Q, stats = evd.eigh_mixed(At, sweeps=sweeps, target=target, b=b, check=check)
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
    assert abs(st[0] - r) <= 1e-3 * r + 1e-18  # the reported residual is the real one
    assert abs(st[1] - scaled_orth(Q)) <= 1e-3 * st[1] + 1e-18
    assert st[2] == 0


@pytest.mark.parametrize("n,seed", [(256, 2), (1024, 3)])
def test_mixed_refined_gaussian(n, seed):
    A = W.gaussian_sym(n, seed=seed, scaled=True)
    w_ref = oracle.syev(A, jobz="N")
    res = []
    for sw in (0, 1, 2, 3):
        w, Q, st = run_mixed(A, sweeps=sw, b=32)
        assert st[2] == sw
        res.append(scaled_res(A, w, Q))
    assert res[2] <= res[0]
    w, Q, st = run_mixed(A, sweeps=8, b=32, target=TARGET)
    assert 1 <= st[2] <= 8
    assert scaled_res(A, w, Q) <= TARGET
    assert scaled_orth(Q) <= TARGET
    assert st[0] <= TARGET and st[1] <= TARGET
    assert M.eig_error(w, w_ref) <= 1e-12
    assert np.all(np.diff(w) >= 0)


def test_mixed_known_spectrum_well_separated():
    n = 600
    A, lam = W.known_spectrum(n, seed=5, spectrum="uniform", reflectors=16)
    w, Q, st = run_mixed(A, sweeps=8, b=32, target=TARGET)
    assert M.eig_error(w, lam) <= 1e-12
    assert scaled_res(A, w, Q) <= TARGET and scaled_orth(Q) <= TARGET


def test_mixed_clustered_spectrum():
    """16 clusters of 8 eigenvalues at relative gaps 1e-8: the clusters are
    resolved by the Rayleigh-Ritz step of the refinement."""
    n = 512
    A, lam = W.known_spectrum(n, seed=8, spectrum="clustered", reflectors=16)
    w, Q, st = run_mixed(A, sweeps=8, b=32, target=TARGET)
    print(f"clustered n={n}: eta={M.eig_error(w, lam):.2e} res={scaled_res(A, w, Q):.2e} "
          f"orth={scaled_orth(Q):.2e} sweeps={st[2]:.0f} clusters={st[4]:.0f} kmax={st[5]:.0f}")
    assert M.eig_error(w, lam) <= 1e-12
    assert scaled_res(A, w, Q) <= TARGET and scaled_orth(Q) <= TARGET
    assert np.all(np.diff(w) >= 0)


@pytest.mark.parametrize("n", [1024, 2048, 4096])
def test_mixed_logspaced_bj_c4_spectrum(n):
    """The mixed workload's spectrum: |lambda| log-spaced over [1e-6, 1] with
    random signs (dense near 0, so most of the spectrum forms one cluster at
    the FP32 start), Q from 64 Householder reflectors.  With the 1e-13 target
    the returned pairs meet the residual, orthogonality and eigenvalue gates
    at the sweep count the call reports, and no sweep makes the
    orthogonality worse than the one before."""
    import torch
    A0, lam = W.known_spectrum_device(n, seed=5, spectrum="logspaced", reflectors=64)
    A = A0.cpu().numpy()
    w, Q, st = run_mixed(A, sweeps=8, b=32 if n < 4096 else 64, target=TARGET)
    res, orth, eta = scaled_res(A, w, Q), scaled_orth(Q), M.eig_error(w, lam)
    print(f"logspaced n={n}: sweeps={st[2]:.0f} res={res:.2e} orth={orth:.2e} eta={eta:.2e} "
          f"delta={st[3]:.2e} clusters={st[4]:.0f} kmax={st[5]:.0f}")
    assert res <= TARGET and orth <= TARGET and eta <= 1e-12
    assert abs(st[0] - res) <= 1e-2 * res + 1e-18
    # sweep by sweep: orthogonality never gets worse
    prev = None
    for sw in range(0, int(st[2]) + 1):
        _, Qk, stk = run_mixed(A, sweeps=sw, b=32 if n < 4096 else 64)
        o = scaled_orth(Qk)
        if prev is not None:
            assert o <= max(prev, 1e-15), (sw, o, prev)
        prev = o
    del torch


def test_mixed_target_missed_reports_status():
    """No sweep allowed but a 1e-13 target: the FP32 pipeline's pairs are
    returned with EVD_ERR_NOT_CONVERGED."""
    from paper_2511_16174_amd import evd
    import torch
    n = 300
    A = W.gaussian_sym(n, seed=9)
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    with pytest.raises(evd.EvdError) as e:
        evd.eigh_mixed(At, sweeps=0, target=TARGET, b=32)
    assert e.value.status == evd.EVD_ERR_NOT_CONVERGED
    # the same call with sweeps allowed meets the target
    w, Q, st = run_mixed(A, sweeps=8, b=32, target=TARGET)
    assert scaled_res(A, w, Q) <= TARGET
