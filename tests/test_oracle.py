"""Pins of the CPU oracle against facts fixed by mathematics, not by itself.

Each pin is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign or index, a transposed operand) fails at least one of them;
``test_planted_mistakes_are_caught`` plants such mistakes in a temporary copy
of ``oracle.c`` and checks that the pins notice.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    vals = [float(x) for x in open(os.path.join(GOLDEN, name)) if x.strip() and not x.startswith("#")]
    return np.array(vals)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 2, 3, 12, 50, 129])
def test_laplacian_closed_form_tridiagonal(n):
    d, e = 2.0 * np.ones(n), -np.ones(n - 1)
    w, Q = oracle.stev(d, e)
    lam = W.laplacian_eigenvalues(n)
    assert np.max(np.abs(w - lam)) <= 8 * n * M.EPS * 4
    # eigenvectors v_k(j) = sqrt(2/(n+1)) sin(j k pi/(n+1)), up to sign; the
    # eigenvalues are simple, so each column is fixed up to sign.
    j = np.arange(1, n + 1)[:, None]
    k = np.arange(1, n + 1)[None, :]
    V = np.sqrt(2.0 / (n + 1)) * np.sin(j * k * np.pi / (n + 1))
    V = V[:, np.argsort(2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))]
    for c in range(n):
        s = np.sign(Q[:, c] @ V[:, c])
        assert np.max(np.abs(Q[:, c] - s * V[:, c])) <= 1e-12


def test_golden_fixtures_closed_forms():
    w = oracle.syev(W.kac_matrix(8), jobz="N")
    assert np.max(np.abs(w - load_golden("kac_n8.txt"))) <= 1e-12
    w = oracle.syev(W.laplacian_1d(12), jobz="N")
    assert np.max(np.abs(w - load_golden("laplacian_n12.txt"))) <= 1e-14
    w = oracle.syev(W.tight_binding(4), jobz="N")
    assert np.max(np.abs(w - load_golden("torus_L4.txt"))) <= 1e-13


@pytest.mark.parametrize("n", [5, 16, 40, 97])
def test_kac_closed_form_dense(n):
    A = W.kac_matrix(n)
    w, Q = oracle.syev(A)
    assert np.max(np.abs(w - W.kac_eigenvalues(n))) <= 1e-11 * n
    assert M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10


@pytest.mark.parametrize("n,seed", [(30, 1), (101, 2), (256, 3)])
def test_rotated_laplacian(n, seed):
    """A = H T H with random reflectors: the full pipeline (tridiagonalization,
    accumulation, QL, sort) must return the closed-form spectrum of T."""
    r = W.rng(seed)
    A = W.apply_reflectors_two_sided(W.laplacian_1d(n), W.reflector_vectors(n, 8, r))
    w, Q = oracle.syev(A)
    assert M.eig_error(w, W.laplacian_eigenvalues(n)) <= 1e-13
    assert M.residual(A, w, Q) <= 10
    assert M.orthogonality(Q) <= 10


@pytest.mark.parametrize("L", [3, 4, 5, 6])
def test_clean_torus_closed_form(L):
    A = W.tight_binding(L)
    w, Q = oracle.syev(A)
    assert M.eig_error(w, W.tight_binding_clean_eigenvalues(L)) <= 1e-13
    assert M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10


def near_tridiagonal_positive(n, delta=1e-20):
    """tridiag(1, 2, 1) plus a 1e-20 entry at (2, 0): the Householder vector of
    column 0 has x_0 = 1 > 0 and a negligible tail, the case where choosing
    beta with the sign of x_0 cancels catastrophically.  Eigenvalues are
    2 + 2 cos(k pi/(n+1)) up to O(delta)."""
    A = 2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    A[2, 0] = A[0, 2] = delta
    k = np.arange(1, n + 1)
    return np.asfortranarray(A), np.sort(2.0 + 2.0 * np.cos(k * np.pi / (n + 1)))


def test_householder_sign_choice_is_stable():
    A, lam = near_tridiagonal_positive(24)
    w, Q = oracle.syev(A)
    assert M.eig_error(w, lam) <= 1e-14
    assert M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10


# ---------------------------------------------------------------- known spectra
@pytest.mark.parametrize("spectrum", ["clustered", "logspaced", "uniform", "geometric", "cluster0", "normal"])
def test_known_spectrum(spectrum):
    n = 300
    A, lam = W.known_spectrum(n, seed=11, spectrum=spectrum, reflectors=16)
    w, Q = oracle.syev(A)
    assert M.eig_error(w, lam) <= 1e-13
    assert M.residual(A, w, Q) <= 10
    assert M.orthogonality(Q) <= 10


# ---------------------------------------------------------------- brute force
def test_jacobi_pinned_by_closed_forms():
    w, V, _ = oracle.jacobi(W.kac_matrix(9))
    assert np.max(np.abs(w - W.kac_eigenvalues(9))) <= 1e-12
    w, V, _ = oracle.jacobi(W.laplacian_1d(20))
    assert np.max(np.abs(w - W.laplacian_eigenvalues(20))) <= 4 * 20 * M.EPS * 4.0
    assert M.residual(W.laplacian_1d(20), w, V) <= 10


@pytest.mark.parametrize("n", [1, 2, 3, 7, 31, 32, 33, 63, 64])
def test_ql_agrees_with_jacobi(n):
    """Two independent algorithms (QL on the tridiagonal form vs Jacobi on the
    dense matrix) on the same random symmetric matrix."""
    A = W.gaussian_sym(n, seed=100 + n)
    w, Q = oracle.syev(A)
    wj, V, _ = oracle.jacobi(A)
    assert M.eig_error(w, wj) <= 1e-14 * max(4, n)
    assert M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10
    assert M.residual(A, wj, V) <= 10 and M.orthogonality(V) <= 10
    # simple, well separated eigenvalues -> eigenvectors agree up to sign
    gaps = np.diff(wj)
    for c in range(n):
        g = min(gaps[c - 1] if c > 0 else np.inf, gaps[c] if c < n - 1 else np.inf)
        if g > 1e-3:
            s = np.sign(Q[:, c] @ V[:, c])
            assert np.linalg.norm(Q[:, c] - s * V[:, c]) <= 1e-10


def test_library_routine_special_case():
    """The plain EVD reduces to LAPACK's symmetric eigensolver (numpy)."""
    A = W.gaussian_sym(200, seed=5)
    w = oracle.syev(A, jobz="N")
    assert M.eig_error(w, np.linalg.eigvalsh(A)) <= 1e-14


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("n", [10, 200])
def test_trace_and_frobenius_invariants(n):
    A = W.gaussian_sym(n, seed=7)
    w = oracle.syev(A, jobz="N")
    assert abs(w.sum() - np.trace(A)) <= 1e-12 * n * np.abs(A).max()
    assert abs((w ** 2).sum() - (A ** 2).sum()) <= 1e-12 * (A ** 2).sum()


def test_tridiag_preserves_spectrum_and_first_column():
    A = W.gaussian_sym(60, seed=9)
    d, e = oracle.tridiag(A)
    w = oracle.stev(d, e, jobz="N")
    assert M.eig_error(w, np.linalg.eigvalsh(A)) <= 1e-14
    # the first diagonal entry is untouched (Q e_1 = e_1)
    assert d[0] == A[0, 0]
    assert abs(abs(e[0]) - np.linalg.norm(A[1:, 0])) <= 1e-13 * np.linalg.norm(A[1:, 0])


# ---------------------------------------------------------------- Sturm count
def test_sturm_counts_exact_on_closed_form():
    n = 64
    d, e = 2.0 * np.ones(n), -np.ones(n - 1)
    lam = W.laplacian_eigenvalues(n)
    mids = 0.5 * (lam[1:] + lam[:-1])
    for i, s in enumerate(mids):
        assert oracle.sturm(d, e, s) == i + 1
    assert oracle.sturm(d, e, lam[0] - 1) == 0
    assert oracle.sturm(d, e, lam[-1] + 1) == n
    # Kac tridiagonal: integer spectrum
    K = W.kac_matrix(11)
    dk, ek = np.diag(K).copy(), np.diag(K, -1).copy()
    for i, v in enumerate(W.kac_eigenvalues(11)):
        assert oracle.sturm(dk, ek, v + 0.5) == i + 1


# ---------------------------------------------------------------- edge cases
def test_edge_cases():
    assert oracle.syev(np.zeros((0, 0)), jobz="N").size == 0
    w, Q = oracle.syev(np.array([[3.5]]))
    assert w[0] == 3.5 and Q[0, 0] == 1.0
    a, b, c = 2.0, 1.0, -1.0
    w = oracle.syev(np.array([[a, b], [b, c]]), jobz="N")
    mid, rad = 0.5 * (a + c), np.hypot(0.5 * (a - c), b)
    assert np.allclose(w, [mid - rad, mid + rad], rtol=0, atol=1e-15)
    D = np.diag([3.0, -1.0, 2.0, 2.0, 0.0])
    w, Q = oracle.syev(D)
    assert np.array_equal(w, np.sort(np.diag(D)))
    Z = np.zeros((6, 6))
    w, Q = oracle.syev(Z)
    assert np.all(w == 0) and M.orthogonality(Q) <= 1
    # block diagonal with exact zero couplings (reflector tau = 0 path)
    B = np.zeros((8, 8))
    B[:4, :4] = W.gaussian_sym(4, 1)
    B[4:, 4:] = W.gaussian_sym(4, 2)
    w, Q = oracle.syev(B)
    assert M.residual(B, w, Q) <= 10 and M.orthogonality(Q) <= 10


def test_uplo_reads_only_one_triangle():
    A = W.gaussian_sym(40, seed=3)
    junk_upper = np.tril(A) + np.triu(np.full_like(A, 1e9), 1)
    junk_lower = np.triu(A) + np.tril(np.full_like(A, -1e9), -1)
    wl = oracle.syev(junk_upper, jobz="N", uplo="L")
    wu = oracle.syev(junk_lower, jobz="N", uplo="U")
    wr = oracle.syev(A, jobz="N")
    assert np.array_equal(wl, wr) and np.array_equal(wu, wr)


# ---------------------------------------------------------------- mutation check
MUTATIONS = {
    "dropped_rank2_term": ("col[i] -= v[i] * wj + p[i] * vj;", "col[i] -= v[i] * wj;"),
    "wrong_sign_beta": ("double beta = (x0 >= 0.0) ? -nrm : nrm;", "double beta = (x0 >= 0.0) ? nrm : -nrm;"),
    "half_factor_dropped": ("const double half = 0.5 * t * pv;", "const double half = t * pv;"),
    "ql_rotation_sign": ("b2_set(B, k + 1, j, s * x + c * y);", "b2_set(B, k + 1, j, s * x - c * y);"),
    "q_accum_index": ("double s = col[0];", "double s = 0.0;"),
    "shift_wrong_corner": ("const double mu = a - bv * bv / (delta + sg * hypot(delta, bv));",
                           "const double mu = c2 - bv * bv / (delta + sg * hypot(delta, bv));"),
    "q_rotation_transposed": ("qa[i] = c * x - s * y;", "qa[i] = c * x + s * y;"),
    "sturm_sign": ("if (q < 0.0) ++cnt;", "if (q > 0.0) ++cnt;"),
    "jacobi_theta_sign": ("const double theta = (aqq - app) / (2.0 * apq);",
                          "const double theta = (app - aqq) / (2.0 * apq);"),
}


def _pins_pass(lib_path):
    """A compact version of the pins above, run against a given oracle build."""
    import ctypes
    saved = oracle._lib
    try:
        oracle._lib = None
        lib = ctypes.CDLL(lib_path)
        real = oracle._LIB
        oracle._LIB = lib_path
        oracle._load()
        oracle._LIB = real
        ok = True
        try:
            A, lam = W.known_spectrum(40, seed=3, spectrum="uniform", reflectors=6)
            w, Q = oracle.syev(A)
            ok &= M.eig_error(w, lam) <= 1e-13 and M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10
            d, e = 2.0 * np.ones(20), -np.ones(19)
            lam = W.laplacian_eigenvalues(20)
            ok &= all(oracle.sturm(d, e, 0.5 * (lam[i] + lam[i + 1])) == i + 1 for i in range(19))
            wj, V, _ = oracle.jacobi(W.kac_matrix(9))
            ok &= np.max(np.abs(wj - W.kac_eigenvalues(9))) <= 1e-12
            A, lam = near_tridiagonal_positive(12)
            w, Q = oracle.syev(A)
            ok &= M.eig_error(w, lam) <= 1e-14 and M.orthogonality(Q) <= 10
        except Exception:
            ok = False
        del lib
        return bool(ok)
    finally:
        oracle._lib = saved


def test_planted_mistakes_are_caught():
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    tmp = tempfile.mkdtemp()
    try:
        clean = os.path.join(tmp, "clean.so")
        cpath = os.path.join(tmp, "clean.c")
        open(cpath, "w").write(src)
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", clean, cpath, "-lm"])
        assert _pins_pass(clean), "the unmutated oracle must pass the pins"
        for name, (old, new) in MUTATIONS.items():
            assert src.count(old) == 1, name
            mpath = os.path.join(tmp, name + ".c")
            open(mpath, "w").write(src.replace(old, new))
            so = os.path.join(tmp, name + ".so")
            subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", so, mpath, "-lm"])
            assert not _pins_pass(so), f"planted mistake '{name}' was not caught"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
