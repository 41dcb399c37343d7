"""Accuracy metrics for an eigendecomposition, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper judges an eigendecomposition by its backward error
||A - Q Lambda Q^T|| / (n ||A||) and its orthogonality ||I - Q Q^T|| / n
(Section 3.3.1 and Table 2).  The norms carry no subscript there; Frobenius
norms are used here, and the ratios are also reported in units of the machine
epsilon eps = 2^-52 (the convention of LAPACK's test ratios):

    rho_res  = ||A Q - Q diag(w)||_F / (n ||A||_F eps)
    rho_orth = ||Q^T Q - I||_F / (n eps)
    eta      = max_i |w_i - w_ref_i| / ||A||_2,  ||A||_2 = max(|w_ref_1|, |w_ref_n|)

The mixed-precision path is accepted on the same two ratios without the eps
(the paper's normalisation of Section 3.3.1): ``scaled_residual`` and
``scaled_orthogonality`` must be <= 1e-13.
"""
from __future__ import annotations

import numpy as np

EPS = float(np.finfo(np.float64).eps)  # 2^-52


def symmetrize(A, uplo: str = "L") -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    L = np.tril(A) if uplo.upper() == "L" else np.triu(A)
    return L + L.T - np.diag(np.diag(A))


def residual(A, w, Q) -> float:
    """||A Q - Q diag(w)||_F / (n ||A||_F eps); A must be the full symmetric matrix."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if n == 0:
        return 0.0
    R = A @ Q - Q * np.asarray(w)[None, :]
    na = np.linalg.norm(A)
    if na == 0.0:
        return float(np.linalg.norm(R) / EPS)
    return float(np.linalg.norm(R) / (n * na * EPS))


def backward_error(A, w, Q) -> float:
    """||A - Q diag(w) Q^T||_F / (n ||A||_F), the paper's Table 2 backward error."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    E = A - (Q * np.asarray(w)[None, :]) @ Q.T
    return float(np.linalg.norm(E) / (n * max(np.linalg.norm(A), 1e-300)))


def scaled_residual(A, w, Q) -> float:
    """||A Q - Q diag(w)||_F / (n ||A||_F) (no eps; A full symmetric)."""
    return residual(A, w, Q) * EPS


def scaled_orthogonality(Q) -> float:
    """||Q^T Q - I||_F / n (no eps)."""
    return orthogonality(Q) * EPS


def orthogonality(Q) -> float:
    """||Q^T Q - I||_F / (n eps)."""
    n = Q.shape[0]
    if n == 0:
        return 0.0
    return float(np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) / (n * EPS))


def eig_error(w, w_ref) -> float:
    """max_i |w_i - w_ref_i| / ||A||_2 with ||A||_2 = max(|w_ref_1|, |w_ref_n|)."""
    w = np.sort(np.asarray(w, dtype=np.float64))
    w_ref = np.sort(np.asarray(w_ref, dtype=np.float64))
    if w.size == 0:
        return 0.0
    scale = max(abs(w_ref[0]), abs(w_ref[-1]))
    if scale == 0.0:
        return float(np.max(np.abs(w - w_ref)))
    return float(np.max(np.abs(w - w_ref)) / scale)
