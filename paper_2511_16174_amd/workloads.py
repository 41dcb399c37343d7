"""Seeded synthetic inputs with the structure of the workloads the solver is
measured on.

This module only draws random numbers and assembles input matrices; it holds
none of the eigensolver's arithmetic, and both the GPU path's tests and the
CPU oracle consume exactly the arrays it returns.  Every generator uses
``numpy.random.Generator(PCG64(seed))`` and draws in the order documented.

The paper measures only on synthetic dense symmetric matrices (Section 5,
Table 1 at n = 49152; Table 2 with six spectrum types at n = 16384).  The
recipes here are:

* :func:`gaussian_sym`        A = (G + G^T)/2, or /(2 sqrt(n)) when ``scaled``
* :func:`known_spectrum`      A = H_1 ... H_r diag(lam) H_r ... H_1 with r
                              random Householder reflectors (exact spectrum lam)
* :func:`clustered_spectrum`  lam uniform in [-1, 1] plus 16 clusters of 8
                              eigenvalues at relative gaps 1e-8
* :func:`logspaced_spectrum`  |lam| log-spaced over [1e-6, 1], random signs
* :func:`table2_spectrum`     the six spectrum types of the paper's Table 2
* :func:`tight_binding_batch` nearest-neighbour Hamiltonians on L x L tori
                              (tight-binding models, Section 1)
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_sym(n: int, seed: int, scaled: bool = False) -> np.ndarray:
    """G ~ N(0,1)^{n x n} (row-major draw order), A = (G + G^T)/2 [/ sqrt(n)]."""
    G = rng(seed).standard_normal((n, n))
    A = G + G.T
    A *= 0.5 / math.sqrt(n) if scaled else 0.5
    return np.asfortranarray(A)


def reflector_vectors(n: int, count: int, r: np.random.Generator) -> np.ndarray:
    """``count`` vectors v_i ~ N(0, I_n), drawn first (as rows)."""
    return r.standard_normal((count, n))


def apply_reflectors_two_sided(D: np.ndarray, V: np.ndarray) -> np.ndarray:
    """A = H_1 ... H_r D H_r ... H_1 with H_i = I - 2 v_i v_i^T / (v_i^T v_i).

    Applied innermost first: A <- H_i A H_i for i = r, ..., 1.  An orthogonal
    similarity keeps the spectrum of D exactly (up to rounding).
    """
    A = np.array(D, dtype=np.float64, order="F")
    for v in V[::-1]:
        v = v / np.linalg.norm(v)
        Av = A @ v
        # H A H = A - 2 v (v^T A) - 2 (A v) v^T + 4 (v^T A v) v v^T
        vAv = float(v @ Av)
        A -= 2.0 * np.outer(v, Av)
        A -= 2.0 * np.outer(Av, v)
        A += 4.0 * vAv * np.outer(v, v)
    A = 0.5 * (A + A.T)
    return np.asfortranarray(A)


def clustered_spectrum(n: int, r: np.random.Generator, clusters: int = 16, size: int = 8,
                       gap: float = 1e-8) -> np.ndarray:
    """16 centres uniform on [-1,-0.1] U [0.1,1], members c (1 + j gap), j = 0..7;
    the remaining n - 128 eigenvalues uniform on [-1, 1]."""
    k = min(clusters, max(n // size, 0))
    mag = r.uniform(0.1, 1.0, size=k)
    sgn = np.where(r.uniform(size=k) < 0.5, -1.0, 1.0)
    centres = sgn * mag
    members = (centres[:, None] * (1.0 + gap * np.arange(size)[None, :])).ravel()
    rest = r.uniform(-1.0, 1.0, size=n - members.size)
    return np.sort(np.concatenate([members, rest]))


def logspaced_spectrum(n: int, r: np.random.Generator) -> np.ndarray:
    """lam_i = s_i 10^{-6 (i-1)/(n-1)}, s_i = +-1 with probability 1/2."""
    i = np.arange(n, dtype=np.float64)
    mag = 10.0 ** (-6.0 * i / max(n - 1, 1))
    s = np.where(r.uniform(size=n) < 0.5, -1.0, 1.0)
    return np.sort(s * mag)


def table2_spectrum(kind: str, n: int, r: np.random.Generator) -> np.ndarray:
    """The six spectrum types of the paper's Table 2 (condition number 1e8 and
    largest eigenvalue 1e6 for the first four)."""
    k = kind.lower()
    if k == "cluster0":
        lam = np.full(n, 1e-2)
        lam[-1] = 1e6
    elif k == "cluster1":
        lam = np.full(n, 1e6)
        lam[0] = 1e-2
    elif k == "geometric":
        lam = 1e6 * (1e-8) ** (np.arange(n) / max(n - 1, 1))
    elif k == "arithmetic":
        lam = np.linspace(1e6, 1e-2, n)
    elif k == "normal":
        lam = r.standard_normal(n)
    elif k == "uniform":
        lam = r.uniform(0.0, 1.0, size=n)
    else:
        raise ValueError(kind)
    return np.sort(lam)


def known_spectrum(n: int, seed: int, spectrum: str = "clustered", reflectors: int = 64):
    """A with an exactly known spectrum: returns (A, lam_sorted).

    Draw order: the ``reflectors`` Householder vectors first, then the
    eigenvalues.  ``spectrum`` is 'clustered', 'logspaced', 'uniform' or one of
    the Table 2 kinds.
    """
    r = rng(seed)
    V = reflector_vectors(n, reflectors, r)
    if spectrum == "clustered":
        lam = clustered_spectrum(n, r)
    elif spectrum == "logspaced":
        lam = logspaced_spectrum(n, r)
    elif spectrum == "uniform":
        lam = np.sort(r.uniform(-1.0, 1.0, size=n))
    else:
        lam = table2_spectrum(spectrum, n, r)
    A = apply_reflectors_two_sided(np.diag(lam), V)
    return A, lam


def known_spectrum_device(n: int, seed: int, spectrum: str = "clustered", reflectors: int = 64,
                          device="cuda"):
    """:func:`known_spectrum` assembled on a GPU: the same PCG64 draws in the
    same order on the host, then the two-sided reflector updates with torch
    FP64 tensor operations on ``device`` (the host assembly takes minutes at
    n = 8192 and beyond).  Returns (A as a torch tensor, lam_sorted numpy)."""
    import torch

    r = rng(seed)
    V = reflector_vectors(n, reflectors, r)
    if spectrum == "clustered":
        lam = clustered_spectrum(n, r)
    elif spectrum == "logspaced":
        lam = logspaced_spectrum(n, r)
    elif spectrum == "uniform":
        lam = np.sort(r.uniform(-1.0, 1.0, size=n))
    else:
        lam = table2_spectrum(spectrum, n, r)
    A = torch.diag(torch.from_numpy(lam).to(device))
    for v in V[::-1]:
        v = torch.from_numpy(v / np.linalg.norm(v)).to(device)
        Av = A @ v
        vAv = float(v @ Av)
        A -= 2.0 * torch.outer(v, Av)
        A -= 2.0 * torch.outer(Av, v)
        A += 4.0 * vAv * torch.outer(v, v)
    A = 0.5 * (A + A.t())
    return A.contiguous(), lam


def laplacian_1d(n: int) -> np.ndarray:
    """tridiag(-1, 2, -1); eigenvalues 2 - 2 cos(k pi/(n+1)), k = 1..n."""
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return np.asfortranarray(A)


def laplacian_eigenvalues(n: int) -> np.ndarray:
    k = np.arange(1, n + 1, dtype=np.float64)
    return np.sort(2.0 - 2.0 * np.cos(k * np.pi / (n + 1)))


def tight_binding(L: int, onsite: np.ndarray | None = None, t: float = -1.0) -> np.ndarray:
    """H on an L x L periodic square lattice, site s = x + L y: H_ss = onsite[s],
    H_ij = t for each of the 4 torus neighbours (accumulated, so L = 2 wraps
    onto the same neighbour twice)."""
    n = L * L
    H = np.zeros((n, n))
    if onsite is not None:
        H[np.arange(n), np.arange(n)] = onsite
    for y in range(L):
        for x in range(L):
            s = x + L * y
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                nb = (x + dx) % L + L * ((y + dy) % L)
                H[nb, s] += t
    return np.asfortranarray(H)


def tight_binding_clean_eigenvalues(L: int, t: float = -1.0) -> np.ndarray:
    """Eigenvalues of the clean (zero on-site) torus: 2t cos(2 pi kx/L) + 2t cos(2 pi ky/L)."""
    k = 2.0 * np.pi * np.arange(L) / L
    lam = 2.0 * t * (np.cos(k)[:, None] + np.cos(k)[None, :])
    return np.sort(lam.ravel())


def tight_binding_batch(count: int, seed: int, lmin: int = 8, lmax: int = 45):
    """``count`` Hamiltonians: L_i ~ U{lmin..lmax} drawn first, then per matrix
    the on-site energies eps ~ U[-2, 2] (n = L^2 of them).  Returns (Ls, mats)."""
    r = rng(seed)
    Ls = r.integers(lmin, lmax + 1, size=count)
    mats = []
    for L in Ls:
        eps = r.uniform(-2.0, 2.0, size=int(L) * int(L))
        mats.append(tight_binding(int(L), eps))
    return [int(L) for L in Ls], mats


def kac_matrix(n: int) -> np.ndarray:
    """Symmetrised Kac-Sylvester-Clement matrix: zero diagonal, off-diagonals
    sqrt(i (n - i)), i = 1..n-1; eigenvalues -(n-1), -(n-3), ..., n-1."""
    off = np.sqrt(np.arange(1, n) * (n - np.arange(1, n)))
    return np.asfortranarray(np.diag(off, 1) + np.diag(off, -1))


def kac_eigenvalues(n: int) -> np.ndarray:
    return np.arange(-(n - 1), n, 2, dtype=np.float64)
