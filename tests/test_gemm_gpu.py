"""FP64 MFMA GEMM vs plain FP64 numpy products (through the C ABI)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.asfortranarray(x).T.copy()).cuda()  # memory = column-major x


def host(t, m, n):
    return t.cpu().numpy().T[:m, :n]


def cm_empty(m, n):
    return torch.zeros((max(n, 1), max(m, 1)), dtype=torch.float64, device="cuda")


CASES = [
    ("N", "N", 0, 1, 1, 1), ("N", "N", 0, 17, 5, 3), ("N", "T", 0, 130, 70, 33), ("T", "N", 0, 64, 64, 64),
    ("T", "T", 0, 129, 257, 100), ("N", "N", 0, 300, 200, 1000), ("S", "N", 0, 200, 64, 200),
    ("S", "T", 0, 333, 40, 333), ("N", "T", 1, 300, 300, 128), ("N", "N", 1, 129, 129, 17),
    ("T", "N", 0, 64, 64, 5000), ("N", "N", 0, 2048, 64, 2048), ("S", "N", 0, 1000, 64, 1000),
]


@pytest.mark.parametrize("opa,opb,lower,m,n,k", CASES)
def test_dgemm_matches_fp64(opa, opb, lower, m, n, k):
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    Ash = (m, k) if opa == "N" else ((k, m) if opa == "T" else (m, m))
    Bsh = (k, n) if opb == "N" else (n, k)
    A = rng.standard_normal(Ash)
    B = rng.standard_normal(Bsh)
    C0 = rng.standard_normal((m, n))
    alpha, beta = -0.75, 0.5
    if opa == "S":
        Afull = np.tril(A) + np.tril(A, -1).T
        A_for = np.tril(A) + np.triu(np.full_like(A, np.nan), 1)  # upper triangle must not be read
        opA = Afull
    else:
        A_for = A
        opA = A if opa == "N" else A.T
    opB = B if opb == "N" else B.T
    ref = alpha * (opA @ opB) + beta * C0
    dA, dB, dC = dev(A_for), dev(B), dev(C0)
    wb = ctx.evd_dgemm_work_size(m, n, k)
    work = torch.empty(max(wb // 8, 1), dtype=torch.float64, device="cuda")
    ctx.evd_dgemm(opa, opb, lower, m, n, k, alpha, dA, A_for.shape[0], dB, B.shape[0], beta, dC, m, work, wb)
    torch.cuda.synchronize()
    out = host(dC, m, n)
    scale = np.abs(opA).max() * np.abs(opB).max() * k + np.abs(C0).max()
    tol = 4 * k * np.finfo(float).eps * scale + 1e-300
    if lower:
        mask = np.tril(np.ones((m, n), bool))
        assert np.max(np.abs(out[mask] - ref[mask])) <= tol
        assert np.array_equal(out[~mask], C0[~mask])  # strict upper untouched
    else:
        assert np.max(np.abs(out - ref)) <= tol


def test_dgemm_no_workspace_equals_splitk():
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    rng = np.random.default_rng(3)
    m, n, k = 64, 64, 8192
    A, B = rng.standard_normal((k, m)), rng.standard_normal((k, n))
    ref = A.T @ B
    for use_ws in (False, True):
        dC = cm_empty(m, n)
        wb = ctx.evd_dgemm_work_size(m, n, k) if use_ws else 0
        work = torch.empty(max(wb // 8, 1), dtype=torch.float64, device="cuda") if use_ws else None
        ctx.evd_dgemm("T", "N", 0, m, n, k, 1.0, dev(A), k, dev(B), k, 0.0, dC, m, work, wb)
        torch.cuda.synchronize()
        assert np.max(np.abs(host(dC, m, n) - ref)) <= 4 * k * 2.2e-16 * 20


@pytest.mark.parametrize("m,n,k,opa,lower,alpha,beta", [(64, 64, 20000, "T", 1, 0.5, 2.0),
                                                        (512, 64, 32768, "T", 0, -1.0, 1.0),
                                                        (300, 64, 5000, "N", 0, 1.0, 0.5),
                                                        (100, 3, 4096, "T", 0, 1.0, 0.0)])
def test_dgemm_many_splits_small_outputs(m, n, k, opa, lower, alpha, beta):
    """Small outputs with long K take many K splits (up to 256) and a split sum
    shared by several lanes per entry; alpha, beta and the lower-triangle
    mode apply to the summed product."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    rng = np.random.default_rng(m + k)
    A = rng.standard_normal((k, m)) if opa == "T" else rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    C0 = rng.standard_normal((m, n))
    opA = A.T if opa == "T" else A
    ref = alpha * (opA @ B) + beta * C0
    dC = dev(C0)
    wb = ctx.evd_dgemm_work_size(m, n, k)
    assert wb > 0
    work = torch.empty(wb // 8 + 1, dtype=torch.float64, device="cuda")
    lda = k if opa == "T" else m
    ctx.evd_dgemm(opa, "N", lower, m, n, k, alpha, dev(A), lda, dev(B), k, beta, dC, m, work, wb)
    torch.cuda.synchronize()
    out = host(dC, m, n)
    tol = 4 * k * 2.2e-16 * np.abs(opA).max() * np.abs(B).max() * abs(alpha) * 4 + 1e-12
    if lower:
        mask = np.tril(np.ones((m, n), bool))
        assert np.max(np.abs(out[mask] - ref[mask])) <= tol
        assert np.array_equal(out[~mask], C0[~mask])
    else:
        assert np.max(np.abs(out - ref)) <= tol


@pytest.mark.parametrize("opa,opb,lower,m,n,k,beta", [
    ("N", "N", 0, 2900, 3001, 640, 0.5), ("T", "N", 0, 3000, 2950, 512, 0.0), ("N", "T", 2, 3001, 3001, 640, 1.0),
    ("N", "T", 1, 2900, 2900, 256, -1.0), ("T", "T", 0, 2950, 2900, 48, 1.0), ("N", "N", 0, 3200, 3200, 4096, 1.0),
    ("N", "N", 0, 2900, 2900, 650, 1.0), ("N", "N", 0, 3000, 64, 3008, 0.0), ("T", "N", 0, 2900, 64, 512, 1.0),
    ("N", "N", 0, 3000, 70, 640, 0.5), ("T", "N", 0, 2900, 64, 1003, 1.0), ("N", "T", 1, 2900, 2900, 77, 0.5),
    ("T", "T", 0, 2950, 2900, 33, 1.0), ("N", "N", 0, 3000, 64, 16, 1.0), ("N", "N", 0, 3000, 64, 20, 0.5),
    ("T", "N", 0, 2900, 64, 9, 1.0), ("T", "N", 0, 3000, 64, 32, 0.0), ("N", "N", 0, 4000, 64, 4000, 0.0)])
def test_dgemm_direct_lds_matches_staged(opa, opb, lower, m, n, k, beta):
    """128 x 128 and 128 x 64 tiles with whole K slices of 16 run the kernel
    whose slices are loaded straight into LDS (tiles crossing the edge of C
    moved back inside it; the m x 64 x m products of SBR included; a partial
    last slice of K zero-filled); it performs the same products in the same order as the main
    loop staged through registers ("gemm_staged" = 1), so both give the same
    bits; a K split (3200^2 x 4096 with workspace) and the lower-triangle
    modes included; K down to one slice, one and a part, and a part only."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    rng = np.random.default_rng(m + 3 * n + k)
    A = rng.standard_normal((m, k) if opa == "N" else (k, m))
    B = rng.standard_normal((k, n) if opb == "N" else (n, k))
    C0 = rng.standard_normal((m, n))
    alpha = -0.75
    dA, dB = dev(A), dev(B)
    wb = ctx.evd_dgemm_work_size(m, n, k)
    work = torch.empty(max(wb // 8, 1), dtype=torch.float64, device="cuda")
    outs = []
    try:
        for staged in (0, 1):
            ctx.set_param("gemm_staged", staged)
            dC = dev(C0)
            ctx.evd_dgemm(opa, opb, lower, m, n, k, alpha, dA, A.shape[0], dB, B.shape[0], beta, dC, m, work, wb)
            torch.cuda.synchronize()
            outs.append(host(dC, m, n))
    finally:
        ctx.set_param("gemm_staged", 0)
    assert np.array_equal(outs[0], outs[1])
    opA = A if opa == "N" else A.T
    opB = B if opb == "N" else B.T
    ref = alpha * (opA @ opB) + beta * C0
    tol = 4 * k * np.finfo(float).eps * np.abs(opA).max() * np.abs(opB).max() * 4 + 1e-12
    if lower:
        mask = np.tril(np.ones((m, n), bool))
        assert np.max(np.abs(outs[0][mask] - ref[mask])) <= tol
        if lower == 2:
            assert np.array_equal(outs[0][~mask], outs[0].T[~mask])
        else:
            assert np.array_equal(outs[0][~mask], C0[~mask])
    else:
        assert np.max(np.abs(outs[0] - ref)) <= tol
