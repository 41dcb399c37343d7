"""Host-CPU divide and conquer (evd_dstedc_host, the paper's placement of the
D&C stage) against the CPU oracle's implicit QL on the same tridiagonals,
closed forms and the metrics' gates.  Runs without a GPU: the entry point
touches no device."""
import ctypes

import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import evd, workloads as W


def host_dc(d, e, compz="I", threads=4):
    lib = evd.load_library()
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = d.shape[0]
    w = np.zeros(max(n, 1))
    Z = np.zeros((max(n, 1), max(n, 1)), order="F") if compz == "I" else None
    info = ctypes.c_int32(-1)
    ptr = lambda a: a.ctypes.data if a is not None and a.size else None
    st = lib.evd_dstedc_host(compz.encode(), n, ptr(d), ptr(e), ptr(w), ptr(Z), max(n, 1), threads,
                             ctypes.addressof(info))
    assert st == evd.EVD_OK
    return w[:n], (Z[:n, :n] if Z is not None else None), info.value


def tridiag_matrix(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def check(d, e, w, Z, w_ref=None):
    T = tridiag_matrix(d, e)
    if w_ref is None:
        w_ref = oracle.stev(d, e, jobz="N")
    assert np.all(np.diff(w) >= 0)
    assert M.eig_error(w, w_ref) <= 1e-12
    if Z is not None:
        assert M.residual(T, w, Z) <= 10, M.residual(T, w, Z)
        assert M.orthogonality(Z) <= 10, M.orthogonality(Z)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 100, 257, 600])
@pytest.mark.parametrize("threads", [1, 4])
def test_random_tridiagonal(n, threads):
    r = W.rng(900 + n)
    d, e = r.standard_normal(n), r.standard_normal(max(n - 1, 0))
    w, Z, info = host_dc(d, e, threads=threads)
    assert info == 0
    check(d, e, w, Z)


def test_laplacian_closed_form():
    n = 400
    d, e = np.full(n, 2.0), np.full(n - 1, -1.0)
    w, Z, info = host_dc(d, e)
    assert info == 0
    check(d, e, w, Z, W.laplacian_eigenvalues(n))
    # eigenvectors against the closed form sqrt(2/(n+1)) sin(j k pi/(n+1)), up to sign
    j = np.arange(1, n + 1)[:, None]
    k = np.arange(1, n + 1)[None, :]
    V = np.sqrt(2.0 / (n + 1)) * np.sin(j * k * np.pi / (n + 1))
    assert np.max(np.abs(np.abs(np.sum(V * Z, axis=0)) - 1.0)) <= 1e-10


@pytest.mark.parametrize("kind", ["glued_wilkinson", "zero_couplings", "constant", "graded"])
def test_deflation_heavy(kind):
    """Tridiagonals where most of the merge work is deflation: glued
    Wilkinson matrices (close eigenvalue pairs), zero couplings (every merge
    fully deflated), a constant diagonal with tiny couplings, and a graded
    diagonal."""
    if kind == "glued_wilkinson":
        m, g = 21, 12
        wd = np.abs(np.arange(m) - (m - 1) / 2.0)
        d = np.tile(wd, g)
        e = np.ones(m * g - 1)
        e[m - 1::m] = 1e-8
    elif kind == "zero_couplings":
        r = W.rng(3)
        d = r.standard_normal(300)
        e = np.zeros(299)
        e[::7] = r.standard_normal(43)
    elif kind == "constant":
        d = np.ones(256)
        e = np.full(255, 1e-14)
    else:
        d = 10.0 ** (-np.arange(200) / 20.0)
        e = 0.1 * np.sqrt(d[:-1] * d[1:])
    w, Z, info = host_dc(d, e)
    assert info == 0
    check(d, e, w, Z)


def test_eigenvalues_only_matches_vectors_mode():
    r = W.rng(11)
    d, e = r.standard_normal(500), r.standard_normal(499)
    wn, _, info = host_dc(d, e, compz="N")
    assert info == 0
    wv, Z, _ = host_dc(d, e, compz="I")
    check(d, e, wn, None)
    assert M.eig_error(wn, wv) <= 1e-12


def test_from_householder_tridiagonalization():
    """The tridiagonal of a dense symmetric matrix (oracle's one-stage
    reduction): the spectrum equals the matrix's."""
    A = W.gaussian_sym(300, seed=12)
    d, e = oracle.tridiag(A)
    w, Z, info = host_dc(d, e)
    assert info == 0
    check(d, e, w, Z, oracle.syev(A, jobz="N"))


def test_argument_checks():
    lib = evd.load_library()
    d = np.zeros(4)
    assert lib.evd_dstedc_host(b"X", 4, d.ctypes.data, d.ctypes.data, d.ctypes.data, None, 4, 1,
                               None) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_dstedc_host(b"I", 4, d.ctypes.data, d.ctypes.data, d.ctypes.data, None, 4, 1,
                               None) == evd.EVD_ERR_INVALID_ARG   # no Z for vectors
    assert lib.evd_dstedc_host(b"N", -1, None, None, None, None, 1, 1, None) == evd.EVD_ERR_INVALID_ARG
    assert lib.evd_dstedc_host(b"N", 0, None, None, None, None, 1, 1, None) == evd.EVD_OK
