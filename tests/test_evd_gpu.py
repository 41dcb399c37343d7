"""End-to-end parity of the GPU eigendecomposition (evd_dsyevd through the C
ABI) with the CPU oracle, closed forms and known spectra.

Gates (per eigendecomposition, eps = 2^-52):
  rho_res  = ||A Q - Q diag(w)||_F / (n ||A||_F eps) <= 10
  rho_orth = ||Q^T Q - I||_F / (n eps)              <= 10
  eta      = max |w - w_ref| / ||A||_2              <= 1e-12
"""
import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import workloads as W
from tests.gpu_helpers import params

pytestmark = pytest.mark.gpu

RES, ORTH, ETA = 10.0, 10.0, 1e-12


def gpu_eigh(A, jobz="V", uplo="L", b=0):
    from paper_2511_16174_amd import evd
    import torch
    At = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    out = evd.eigh(At, jobz=jobz, uplo=uplo, b=b)
    torch.cuda.synchronize()
    if jobz == "V":
        w, Q = out
        return w.cpu().numpy(), Q.cpu().numpy()
    return out.cpu().numpy(), None


def check(A, w, Q, w_ref):
    assert np.all(np.diff(w) >= 0), "eigenvalues must be ascending"
    eta = M.eig_error(w, w_ref)
    assert eta <= ETA, eta
    if Q is not None:
        res, orth = M.residual(A, w, Q), M.orthogonality(Q)
        assert res <= RES, res
        assert orth <= ORTH, orth


def test_config_n512_b32_vs_oracle():
    """Plain FP64 EVD with vectors, n = 512, A = (G + G^T)/2, b = 32."""
    A = W.gaussian_sym(512, seed=1)
    w, Q = gpu_eigh(A, b=32)
    w_ref, Q_ref = oracle.syev(A)
    check(A, w, Q, w_ref)
    # eigenvectors of well separated eigenvalues agree up to sign (Davis-Kahan)
    gaps = np.minimum(np.r_[np.inf, np.diff(w_ref)], np.r_[np.diff(w_ref), np.inf])
    norm2 = max(abs(w_ref[0]), abs(w_ref[-1]))
    for c in np.where(gaps >= 1e-6 * norm2)[0]:
        s = np.sign(Q[:, c] @ Q_ref[:, c])
        assert np.linalg.norm(Q[:, c] - s * Q_ref[:, c]) <= 100 * np.sqrt(512) * M.EPS * norm2 / gaps[c]


@pytest.mark.parametrize("n,b", [(2, 0), (3, 0), (5, 4), (31, 8), (33, 16), (63, 32), (64, 32), (65, 64),
                                 (100, 4), (129, 64), (257, 16), (300, 2), (700, 64)])
def test_sizes_and_bands(n, b):
    A = W.gaussian_sym(n, seed=10 + n)
    w, Q = gpu_eigh(A, b=b)
    check(A, w, Q, oracle.syev(A, jobz="N"))


def test_n1():
    A = np.array([[-2.5]])
    w, Q = gpu_eigh(A)
    assert w[0] == -2.5 and Q[0, 0] == 1.0


@pytest.mark.parametrize("n", [100, 512])
def test_values_only(n):
    A = W.gaussian_sym(n, seed=3)
    w, _ = gpu_eigh(A, jobz="N")
    check(A, w, None, oracle.syev(A, jobz="N"))


def test_uplo_upper():
    A = W.gaussian_sym(200, seed=8)
    junk = np.triu(A) + np.tril(np.full_like(A, 3e7), -1)
    w, Q = gpu_eigh(junk, uplo="U", b=16)
    check(A, w, Q, oracle.syev(A, jobz="N"))


@pytest.mark.parametrize("spectrum", ["clustered", "logspaced", "geometric", "cluster0", "cluster1"])
def test_known_spectra(spectrum):
    n = 600
    A, lam = W.known_spectrum(n, seed=4, spectrum=spectrum, reflectors=16)
    w, Q = gpu_eigh(A, b=32)
    check(A, w, Q, lam)


@pytest.mark.parametrize("L", [6, 8, 11])
def test_clean_torus_degenerate(L):
    A = W.tight_binding(L)
    w, Q = gpu_eigh(A, b=16)
    check(A, w, Q, W.tight_binding_clean_eigenvalues(L))


def test_rotated_laplacian_closed_form():
    n = 400
    A = W.apply_reflectors_two_sided(W.laplacian_1d(n), W.reflector_vectors(n, 8, W.rng(12)))
    w, Q = gpu_eigh(A, b=32)
    check(A, w, Q, W.laplacian_eigenvalues(n))


def test_trace_frobenius_invariants():
    A = W.gaussian_sym(800, seed=21, scaled=True)
    w, _ = gpu_eigh(A, jobz="N")
    assert abs(w.sum() - np.trace(A)) <= 1e-12 * 800
    assert abs((w ** 2).sum() - (A ** 2).sum()) <= 1e-12 * (A ** 2).sum()


@pytest.mark.parametrize("n,b", [(5, 4), (130, 8), (300, 32), (700, 64), (1000, 32)])
def test_conventional_stage_order(n, b):
    """order = 1: Q = Q_s (H_1 ... H_m Q_d) with the reverse-order BC-back and
    SBR-back applied from the left; same gates as the reordered stages."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    assert ctx.get_param("order") == 1   # the library default
    A = W.gaussian_sym(n, seed=n + 3 * b)
    with params(ctx, order=1):
        w, Q = gpu_eigh(A, b=b)
    check(A, w, Q, oracle.syev(A, jobz="N"))


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("n,b,sub,rt", [(300, 16, 0, 0), (515, 32, 0, 0), (700, 64, 0, 0), (1100, 64, 64, 0),
                                        (700, 64, 16, 0), (1100, 64, 32, 0), (1100, 64, 32, 2), (700, 64, 16, 2)])
def test_blocked_bcback_matches_reflector_by_reflector(n, b, sub, rt, order):
    """The blocked BC-back on the matrix cores (groups of sweeps in compact
    WY; at b = 64 also as 16-sweep block reflectors, "bcback_sub", with one or
    two 16-row tiles per wavefront, "bcback_rt") and the reflector-by-reflector
    kernel give the same eigenvectors up to rounding, in both stage orders."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    A = W.gaussian_sym(n, seed=n + b + order)
    out = []
    for valu in (0, 1):
        with params(ctx, order=order, bcback_valu=valu, bcback_sub=sub, bcback_rt=rt):
            out.append(gpu_eigh(A, b=b))
    (w0, Q0), (w1, Q1) = out
    assert np.array_equal(w0, w1)
    assert np.abs(Q0 - Q1).max() <= 1e-12
    check(A, w0, Q0, oracle.syev(A, jobz="N"))


def solve_device(ctx, A0, jobz="V", b=64):
    """evd_dsyevd on a copy of the device matrix A0 (symmetric, so row- and
    column-major agree): returns (w, X) with X[:, j] the j-th eigenvector."""
    import torch
    n = A0.shape[0]
    A = A0.clone()
    w = torch.empty(n, dtype=torch.float64, device=A0.device)
    info = torch.zeros(1, dtype=torch.int32, device=A0.device)
    with params(ctx, b=b):
        wb = ctx.evd_dsyevd_work_size(jobz, "L", n, n)
        work = torch.empty(wb // 8 + 64, dtype=torch.float64, device=A0.device)
        ctx.evd_dsyevd(jobz, "L", n, A, n, w, work, wb, info)
        torch.cuda.synchronize()
    del work
    assert int(info.item()) == 0
    assert bool((w[1:] >= w[:-1]).all())
    return w, A.t()


@pytest.mark.parametrize("order", [0, 1])
def test_bj_c2_known_clustered_n8192(order):
    """Plain FP64 EVD with vectors at n = 8192, b = 64, on the known spectrum
    (seed 2): 64 random Householder reflectors around diag(lam), lam uniform on
    [-1, 1] plus 16 clusters of 8 eigenvalues at relative gaps 1e-8.  Both
    stage orders; eta against the lam the matrix was built from, rho_res and
    rho_orth of all pairs with torch FP64 products."""
    import torch
    from paper_2511_16174_amd import evd
    from tests.gpu_helpers import device_ratios
    n = 8192
    ctx = evd.context(0)
    A0, lam = W.known_spectrum_device(n, seed=2, spectrum="clustered", reflectors=64)
    with params(ctx, order=order):
        w, X = solve_device(ctx, A0, b=64)
    eta = M.eig_error(w.cpu().numpy(), lam)
    res, orth = device_ratios(A0, w, X)
    print(f"BJ.c2 n={n} order={order}: eta={eta:.2e} rho_res={res:.3f} rho_orth={orth:.3f}")
    assert eta <= ETA, eta
    assert res <= RES, res
    assert orth <= ORTH, orth


FULL_CASES = [("gaussian", 0), ("gaussian", 1), ("uniform", 1)]


@pytest.mark.parametrize("kind,order", FULL_CASES)
def test_full_size_n32768(kind, order):
    """The plain FP64 EVD with vectors at n = 32768, b = 64, in both stage
    orders (order 1, the default, is what the benchmark times).
    'gaussian': A = (G + G^T)/(2 sqrt n) generated on the GPU (the benchmark's
    matrix); 'uniform': 64 reflectors around diag(lam), lam uniform on
    [-1, 1] (seed 3), so eta is checked against the known lam.
    Gates: 48 sampled pairs meet ||A x_j - w_j x_j||_2 / (n ||A||_2 eps) <= 10
    and are orthonormal against every returned vector; the eigenvalues keep
    the trace; eta <= 1e-12 where lam is known."""
    import torch
    from paper_2511_16174_amd import evd
    n = 32768
    dev = torch.device("cuda:0")
    ctx = evd.context(0)
    lam = None
    if kind == "gaussian":
        g = torch.Generator(device=dev)
        g.manual_seed(3)
        G = torch.randn((n, n), dtype=torch.float64, device=dev, generator=g)
        A0 = (G + G.t()) * (0.5 / n ** 0.5)
        del G
    else:
        A0, lam = W.known_spectrum_device(n, seed=3, spectrum="uniform", reflectors=64)
    with params(ctx, order=order):
        w, X = solve_device(ctx, A0, b=64)
    J = torch.randperm(n, generator=torch.Generator().manual_seed(5))[:48].to(dev)
    J[:3] = torch.tensor([0, n // 2, n - 1], device=dev)
    Xs = X[:, J].contiguous()
    norm2 = max(abs(w[0].item()), abs(w[-1].item()))
    res = torch.linalg.norm(A0 @ Xs - Xs * w[J][None, :], dim=0) / (n * norm2 * M.EPS)
    O = X.t() @ Xs
    O[J, torch.arange(J.numel(), device=dev)] -= 1.0
    orth = torch.linalg.norm(O, dim=0).max().item() / (n * M.EPS)
    eta = M.eig_error(w.cpu().numpy(), lam) if lam is not None else float("nan")
    print(f"n={n} {kind} order={order}: max rho_res(col)={res.max().item():.3f} "
          f"max rho_orth(col)={orth:.3f} eta={eta:.2e}")
    assert res.max().item() <= RES, res.max().item()
    assert orth <= ORTH
    assert abs(w.sum().item() - torch.trace(A0).item()) <= 1e-12 * n * norm2
    if lam is not None:
        assert eta <= ETA, eta


def raw_dsyevd(ctx, A, jobz="V", uplo="L"):
    """evd_dsyevd on a host matrix without raising on the device status:
    returns (w, Q or None, info)."""
    import torch
    n = A.shape[0]
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()   # column-major
    w = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    wb = ctx.evd_dsyevd_work_size(jobz, uplo, n, max(n, 1))
    work = torch.empty(max(wb, 256) // 8 + 32, dtype=torch.float64, device="cuda")
    ctx.evd_dsyevd(jobz, uplo, n, Ad, max(n, 1), w, work, wb, info)
    torch.cuda.synchronize()
    Q = Ad.cpu().numpy().T if jobz == "V" else None
    return w.cpu().numpy()[:n], Q, int(info.item())


@pytest.mark.parametrize("n", [1, 2, 100, 300])
@pytest.mark.parametrize("jobz", ["N", "V"])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_input_reports_status(n, jobz, bad):
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    A = W.gaussian_sym(n, seed=40 + n)
    A[n - 1, n // 2] = bad        # lower triangle, referenced by uplo = 'L'
    w, Q, info = raw_dsyevd(ctx, A, jobz=jobz, uplo="L")
    assert info == evd.EVD_ERR_NONFINITE
    assert np.all(np.isnan(w))
    if jobz == "V":
        assert np.all(np.isnan(Q))
    # the next call on the same context and a finite matrix is unaffected
    B = W.gaussian_sym(n, seed=41 + n)
    w, Q, info = raw_dsyevd(ctx, B, jobz=jobz)
    assert info == 0
    check(B, w, Q, oracle.syev(B, jobz="N"))


@pytest.mark.parametrize("row,col", [(2999, 5), (2000, 1000), (1300, 1000), (1600, 1000), (1029, 5), (2999, 2998)])
def test_nonfinite_deep_in_a_long_column(row, col):
    """Entries at every position of the scan's four loads in flight per
    thread and past its first pass over 1024 rows."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    n = 3000
    A = W.gaussian_sym(n, seed=45)
    A[row, col] = np.inf
    w, _, info = raw_dsyevd(ctx, A, jobz="N", uplo="L")
    assert info == evd.EVD_ERR_NONFINITE
    assert np.all(np.isnan(w))


@pytest.mark.parametrize("uplo", ["L", "U"])
def test_nonfinite_entries_outside_the_referenced_triangle_are_ignored(uplo):
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    n = 150
    A = W.gaussian_sym(n, seed=44)
    junk = A.copy()
    if uplo == "L":
        junk[np.triu_indices(n, 1)] = np.nan
        junk[0, n - 1] = np.inf
    else:
        junk[np.tril_indices(n, -1)] = -np.inf
    w, Q, info = raw_dsyevd(ctx, junk, uplo=uplo)
    assert info == 0
    check(A, w, Q, oracle.syev(A, jobz="N"))


def test_zero_matrix():
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    n = 200
    w, Q, info = raw_dsyevd(ctx, np.zeros((n, n)))
    assert info == 0 and np.all(w == 0.0)
    assert M.orthogonality(Q) <= ORTH


def test_forced_dc_nonconvergence_reports_status():
    """One secular iteration per root ("dc_max_iter" = 1) cannot converge:
    the status word says so, and the context works normally afterwards."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    A = W.gaussian_sym(300, seed=45)
    with params(ctx, dc_max_iter=1):
        _, _, info = raw_dsyevd(ctx, A)
    assert info == evd.EVD_ERR_NOT_CONVERGED
    w, Q, info = raw_dsyevd(ctx, A)
    assert info == 0
    check(A, w, Q, oracle.syev(A, jobz="N"))


@pytest.mark.parametrize("n,b,jobz", [(300, 32, "V"), (1000, 32, "V"), (2100, 64, "V"), (2100, 64, "N"),
                                      (8192, 64, "V")])
def test_bc_beside_sbr_matches_bc_after_sbr(n, b, jobz):
    """Bulge chasing started beside SBR ("bc_overlap" = 1, gated by the band
    columns SBR publishes panel by panel) computes exactly what it computes
    after SBR: eigenvalues and eigenvectors agree bit for bit, and both meet
    the oracle's gates."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    A = W.gaussian_sym(n, seed=70 + n + b)
    out = []
    for ov in (0, 1):
        with params(ctx, bc_overlap=ov, b=b):
            w, Q, info = raw_dsyevd(ctx, A, jobz=jobz)
        assert info == 0
        out.append((w, Q))
    (w0, Q0), (w1, Q1) = out
    assert np.array_equal(w0, w1)
    if jobz == "V":
        assert np.array_equal(Q0, Q1)
        if n <= 2100:
            check(A, w1, Q1, oracle.syev(A, jobz="N"))
    else:
        assert M.eig_error(w1, oracle.syev(A, jobz="N")) <= ETA


@pytest.mark.parametrize("jobz", ["N", "V"])
def test_bc_wait_timeout_reports_status(jobz):
    """"debug_gate" makes bulge chasing wait for band columns that are never
    published, with a 2 ms limit: every workgroup leaves, the call reports
    EVD_ERR_TIMEOUT with NaN outputs, and the context works normally
    afterwards."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    n = 700
    A = W.gaussian_sym(n, seed=77)
    with params(ctx, debug_gate=1, spin_limit_ms=2):
        w, Q, info = raw_dsyevd(ctx, A, jobz=jobz)
    assert info == evd.EVD_ERR_TIMEOUT
    assert np.all(np.isnan(w))
    if jobz == "V":
        assert np.all(np.isnan(Q))
    w, Q, info = raw_dsyevd(ctx, A, jobz=jobz)
    assert info == 0
    if jobz == "V":
        check(A, w, Q, oracle.syev(A, jobz="N"))


@pytest.mark.parametrize("n,b", [(300, 32), (1500, 64)])
def test_host_dc_beside_gpu_back_transform(n, b):
    """"dc_host" = 1: D&C on the host CPU in a thread while the GPU forms
    Q_s H_1 ... H_m, then Q = (Q_s H_1 ... H_m) Q_d: the oracle's gates, and
    the eigenvalues agree with the GPU D&C's to 1e-12."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    A = W.gaussian_sym(n, seed=80 + n)
    with params(ctx, dc_host=1, b=b):
        w, Q, info = raw_dsyevd(ctx, A)
    assert info == 0
    check(A, w, Q, oracle.syev(A, jobz="N"))
    with params(ctx, b=b):
        w_gpu, _, _ = raw_dsyevd(ctx, A)
    assert M.eig_error(w, w_gpu) <= 1e-12
