"""Pins of the accuracy metrics in the rejecting direction.

Every parity gate rests on ``oracle.metrics``; a metric that is too lenient
(an extra 1/n, a norm over the wrong axis, a missing square root) would let
wrong results pass silently.  Each test below plants a defect of known size
in an exact eigendecomposition and checks that the metric reports exactly the
magnitude the defect has in closed form, and that the gate then fails.

The exact decomposition is A = Q diag(lam) Q^T with Q a product of random
Householder reflectors (orthogonal up to rounding, so the unperturbed metrics
are O(1) in units of eps and the planted values are many orders above them).

Closed forms used (Q orthogonal, G a plane rotation by theta in columns i, j,
s = sin theta, d = lam_i - lam_j):
  ||A (QG) - (QG) diag(lam)||_F = sqrt(2) |s| |d|
  ||A - (QG) diag(lam) (QG)^T||_F = sqrt(2) |s| |d|
  ||A Q - Q diag(lam + delta e_k)||_F = |delta|
  ||(Q(I + a e_i e_j^T))^T (Q(I + a e_i e_j^T)) - I||_F = sqrt(2 a^2 + a^4)
  ||(Q D)^T (Q D) - I||_F = |2 b + b^2| for D = I + b e_k e_k^T
"""
import math

import numpy as np
import pytest

import oracle.metrics as M
from paper_2511_16174_amd import workloads as W

N = 40


def exact_pair(seed=3, negative_dominant=False):
    r = W.rng(seed)
    lam = np.sort(r.uniform(-1.0, 1.0, size=N))
    if negative_dominant:
        lam[0] = -3.0   # ||A||_2 comes from the negative end
    Q = np.eye(N)
    for v in W.reflector_vectors(N, 6, r):
        v = v / np.linalg.norm(v)
        Q = Q - 2.0 * np.outer(Q @ v, v)
    A = (Q * lam[None, :]) @ Q.T
    A = 0.5 * (A + A.T)
    return A, lam, Q


def rotate(Q, i, j, theta):
    G = np.eye(Q.shape[1])
    c, s = math.cos(theta), math.sin(theta)
    G[i, i] = G[j, j] = c
    G[i, j], G[j, i] = s, -s
    return Q @ G


def test_unperturbed_pair_passes():
    A, lam, Q = exact_pair()
    assert M.residual(A, lam, Q) <= 10
    assert M.orthogonality(Q) <= 10
    assert M.eig_error(lam, lam) == 0.0
    assert M.scaled_residual(A, lam, Q) <= 1e-15
    assert M.scaled_orthogonality(Q) <= 1e-15


@pytest.mark.parametrize("i,j,theta", [(3, 17, 1e-8), (0, N - 1, 3e-9), (10, 11, 1e-6)])
def test_residual_reports_a_rotated_pair(i, j, theta):
    A, lam, Q = exact_pair()
    Qr = rotate(Q, i, j, theta)
    exact = math.sqrt(2.0) * abs(math.sin(theta)) * abs(lam[i] - lam[j])
    nA = np.linalg.norm(lam)
    want = exact / (N * nA * M.EPS)
    got = M.residual(A, lam, Qr)
    assert abs(got - want) <= 1e-4 * want + 2.0, (got, want)
    assert got > 10
    # the unscaled form (the mixed path's 1e-13 acceptance) and the paper's
    # backward error report the same defect without the eps
    assert abs(M.scaled_residual(A, lam, Qr) - want * M.EPS) <= 1e-4 * want * M.EPS + 1e-15
    want_b = exact / (N * nA)
    assert abs(M.backward_error(A, lam, Qr) - want_b) <= 1e-4 * want_b + 1e-15
    # a rotation keeps the basis orthonormal: orthogonality must not flag it
    assert M.orthogonality(Qr) <= 10


@pytest.mark.parametrize("k,delta", [(0, 1e-9), (N // 2, -4e-10), (N - 1, 2.5e-11)])
def test_residual_and_eig_error_report_a_shifted_eigenvalue(k, delta):
    A, lam, Q = exact_pair(negative_dominant=True)
    w = lam.copy()
    w[k] += delta
    want = abs(delta) / (N * np.linalg.norm(lam) * M.EPS)
    got = M.residual(A, w, Q)
    assert abs(got - want) <= 1e-4 * want + 2.0, (got, want)
    assert got > 10
    # eta normalises by ||A||_2 = max(|lam_1|, |lam_n|) = 3 here
    eta = M.eig_error(w, lam)
    assert abs(eta - abs(delta) / 3.0) <= 1e-6 * abs(delta), (eta, delta)
    assert eta > 1e-12


@pytest.mark.parametrize("i,j,a", [(2, 30, 1e-10), (7, 8, 3e-12), (5, 5, 1e-11)])
def test_orthogonality_reports_a_sheared_basis(i, j, a):
    _, _, Q = exact_pair()
    S = np.eye(N)
    S[i, j] += a
    Qs = Q @ S
    if i == j:   # a scaled column: (1 + a)^2 - 1 on one diagonal entry
        exact = abs(2 * a + a * a)
    else:
        exact = math.sqrt(2 * a * a + a ** 4)
    want = exact / (N * M.EPS)
    got = M.orthogonality(Qs)
    assert abs(got - want) <= 1e-3 * want + 2.0, (got, want)
    assert got > 10
    assert abs(M.scaled_orthogonality(Qs) - exact / N) <= 1e-3 * exact / N + 1e-16


def test_eig_error_compares_sorted_values_and_uses_two_norm():
    _, lam, _ = exact_pair(negative_dominant=True)
    w = lam[::-1].copy()   # order must not matter (both are sorted)
    assert M.eig_error(w, lam) == 0.0
    w = lam.copy()
    w[5] = lam[5] + 1e-6
    assert abs(M.eig_error(w, lam) - 1e-6 / 3.0) <= 1e-12
    # the normaliser is ||A||_2, not ||A||_F: on lam = diag(1, ..., 1, 1) the
    # two differ by sqrt(n)
    ones = np.ones(16)
    w = ones.copy()
    w[0] += 1e-8
    assert abs(M.eig_error(w, ones) - 1e-8) <= 1e-15


def test_symmetrize_reads_one_triangle():
    A, _, _ = exact_pair()
    junk = np.tril(A) + np.triu(np.full_like(A, 7e5), 1)
    assert np.array_equal(M.symmetrize(junk, "L"), A * 0 + np.tril(A) + np.tril(A, -1).T)
    junk = np.triu(A) + np.tril(np.full_like(A, 7e5), -1)
    assert np.array_equal(M.symmetrize(junk, "U"), np.triu(A) + np.triu(A, 1).T)


# ---------------------------------------------------------------- mutations
MUTATIONS = [
    # (description, original text, mutated text)
    ("extra 1/n in the residual", "(n * na * EPS)", "(n * n * na * EPS)"),
    ("spectral instead of Frobenius residual norm",
     "return float(np.linalg.norm(R) / (n * na * EPS))", "return float(np.linalg.norm(R, 2) / (n * na * EPS))"),
    ("eigenvalues scale rows instead of columns", "R = A @ Q - Q * np.asarray(w)[None, :]",
     "R = A @ Q - Q * np.asarray(w)[:, None]"),
    ("extra 1/n in the orthogonality", "/ (n * EPS))", "/ (n * n * EPS))"),
    ("orthogonality without the identity", "np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1]))",
     "np.linalg.norm(Q.T @ Q) - math.sqrt(Q.shape[1])"),
    ("eta normalised by the Frobenius norm", "scale = max(abs(w_ref[0]), abs(w_ref[-1]))",
     "scale = float(np.linalg.norm(w_ref))"),
    ("eta as a mean instead of a max", "return float(np.max(np.abs(w - w_ref)) / scale)",
     "return float(np.mean(np.abs(w - w_ref)) / scale)"),
    ("backward error with a transposed factor", "E = A - (Q * np.asarray(w)[None, :]) @ Q.T",
     "E = A - (Q * np.asarray(w)[None, :]) @ Q"),
    ("backward error without 1/n", "/ (n * max(np.linalg.norm(A), 1e-300))",
     "/ max(np.linalg.norm(A), 1e-300)"),
]

PIN_TESTS = [
    (test_unperturbed_pair_passes, [()]),
    (test_residual_reports_a_rotated_pair, [(3, 17, 1e-8), (10, 11, 1e-6)]),
    (test_residual_and_eig_error_report_a_shifted_eigenvalue, [(0, 1e-9), (N // 2, -4e-10)]),
    (test_orthogonality_reports_a_sheared_basis, [(2, 30, 1e-10), (5, 5, 1e-11)]),
    (test_eig_error_compares_sorted_values_and_uses_two_norm, [()]),
]


def test_planted_metric_mistakes_are_caught(monkeypatch, tmp_path):
    import importlib.util
    import inspect
    src = inspect.getsource(M)
    for what, old, new in MUTATIONS:
        assert src.count(old) == 1, f"mutation anchor not found: {what}"
        path = tmp_path / "mutated_metrics.py"
        mutated = src.replace(old, new).replace("from __future__ import annotations\n",
                                                "from __future__ import annotations\nimport math\n", 1)
        path.write_text(mutated)
        spec = importlib.util.spec_from_file_location("mutated_metrics", path)
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        caught = False
        with monkeypatch.context() as mp:
            for name in ("residual", "orthogonality", "eig_error", "backward_error", "scaled_residual",
                         "scaled_orthogonality", "symmetrize"):
                mp.setattr(M, name, getattr(mod, name))
            for fn, cases in PIN_TESTS:
                for args in cases:
                    try:
                        fn(*args)
                    except (AssertionError, ValueError, FloatingPointError):
                        caught = True
                        break
                if caught:
                    break
        assert caught, f"planted mistake not caught: {what}"
