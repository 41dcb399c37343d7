"""CPU oracle for the dense symmetric eigendecomposition A = Q diag(w) Q^T.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and nothing here falls back to the GPU path.

The arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP over whole rows or
columns); this module only marshals numpy arrays into it.  Functions:

* :func:`syev`      -- one-stage Householder tridiagonalization + implicit QL
                       (the plain definition of the result the paper's
                       two-stage method reaches; paper Section 1, Algorithm 1
                       ENSURE clause)
* :func:`tridiag`   -- the tridiagonalization alone (d, e)
* :func:`stev`      -- eigenpairs of a symmetric tridiagonal matrix (QL)
* :func:`jacobi`    -- cyclic Jacobi, an independent brute force for small n
* :func:`sturm`     -- Sturm count #{eig(T) < sigma}

The metrics the paper uses to judge an eigendecomposition (Section 3.3.1,
Table 2: backward error and orthogonality) are in :mod:`oracle.metrics`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i64, dp, c = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_char
    lib.oracle_tridiag.argtypes = [i64, dp, i64, dp, dp, dp]
    lib.oracle_form_q.argtypes = [i64, dp, i64, dp, dp, i64]
    lib.oracle_ql.argtypes = [i64, dp, dp, dp, i64]
    lib.oracle_sort.argtypes = [i64, dp, dp, i64]
    lib.oracle_syev.argtypes = [c, i64, dp, i64, dp, dp, i64]
    lib.oracle_stev.argtypes = [i64, dp, dp, dp, dp, i64]
    lib.oracle_jacobi.argtypes = [i64, dp, i64, dp, dp, i64, ctypes.c_int]
    lib.oracle_sturm.argtypes = [i64, dp, dp, ctypes.c_double]
    lib.oracle_sturm.restype = i64
    lib.oracle_num_threads.restype = ctypes.c_int
    for f in ("oracle_tridiag", "oracle_form_q", "oracle_ql", "oracle_sort", "oracle_syev",
              "oracle_stev", "oracle_jacobi"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fortran(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def syev(A, jobz: str = "V", uplo: str = "L"):
    """Eigenvalues (ascending) and, for jobz='V', orthonormal eigenvectors.

    Only the ``uplo`` triangle of ``A`` is read.  Returns ``w`` or ``(w, Q)``.
    """
    A = _fortran(A)
    n = A.shape[0]
    w = np.zeros(n)
    Q = np.zeros((n, n), order="F") if jobz.upper() == "V" else None
    info = _load().oracle_syev(uplo.encode()[:1], n, _p(A), max(n, 1), _p(w),
                               _p(Q) if Q is not None else None, max(n, 1))
    if info != 0:
        raise RuntimeError(f"oracle_syev failed, info={info}")
    return (w, Q) if Q is not None else w


def tridiag(A):
    """Householder tridiagonalization of the full symmetric A: returns (d, e)."""
    S = _fortran(A).copy(order="F")
    n = S.shape[0]
    d, e, tau = np.zeros(n), np.zeros(max(n, 1)), np.zeros(max(n, 1))
    _load().oracle_tridiag(n, _p(S), max(n, 1), _p(d), _p(e), _p(tau))
    return d, e[: max(n - 1, 0)]


def stev(d, e, jobz: str = "V"):
    """Eigenpairs of the symmetric tridiagonal matrix tridiag(e, d, e)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    n = d.shape[0]
    e = np.ascontiguousarray(np.concatenate([np.asarray(e, dtype=np.float64), [0.0]])[: max(n, 1)])
    w = np.zeros(n)
    Q = np.zeros((n, n), order="F") if jobz.upper() == "V" else None
    info = _load().oracle_stev(n, _p(d), _p(e), _p(w), _p(Q) if Q is not None else None, max(n, 1))
    if info != 0:
        raise RuntimeError(f"oracle_stev failed, info={info}")
    return (w, Q) if Q is not None else w


def jacobi(A, max_sweeps: int = 50):
    """Cyclic-by-row Jacobi on the full symmetric A: returns (w, V, sweeps)."""
    S = _fortran(A).copy(order="F")
    n = S.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), order="F")
    sweeps = _load().oracle_jacobi(n, _p(S), max(n, 1), _p(w), _p(V), max(n, 1), max_sweeps)
    if sweeps < 0:
        raise RuntimeError("oracle_jacobi did not converge")
    return w, V, sweeps


def sturm(d, e, sigma: float) -> int:
    """Number of eigenvalues of tridiag(e, d, e) strictly below sigma."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(np.concatenate([np.asarray(e, dtype=np.float64), [0.0]]))
    return int(_load().oracle_sturm(d.shape[0], _p(d), _p(e), float(sigma)))
