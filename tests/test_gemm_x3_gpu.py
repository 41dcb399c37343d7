"""Split-BF16x3 FP32 GEMM vs an FP64 product: componentwise error within
(3 * 2^-17 + k * 2^-24) * (|A| |B|)_ij (split error of the dropped lo*lo term
and of the bf16 rounding of each part, plus FP32 accumulation)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev32(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.float32).T)).cuda()


def host32(t, m, n):
    return t.cpu().numpy().astype(np.float64).reshape(-1)[: m * n].reshape(n, m).T


@pytest.mark.parametrize("opa,opb,lower,m,n,k", [
    ("N", "N", 0, 1, 1, 1), ("N", "N", 0, 33, 17, 45), ("N", "T", 0, 300, 200, 129), ("T", "N", 0, 64, 64, 4096),
    ("T", "T", 0, 130, 257, 70), ("S", "N", 0, 500, 64, 500), ("N", "T", 1, 400, 400, 128), ("N", "N", 0, 1024, 1024, 1024),
])
def test_sgemm_x3_error_bound(opa, opb, lower, m, n, k):
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    rng = np.random.default_rng(m + n + k)
    Ash = (m, k) if opa == "N" else ((k, m) if opa == "T" else (m, m))
    Bsh = (k, n) if opb == "N" else (n, k)
    A = rng.standard_normal(Ash).astype(np.float32).astype(np.float64)
    B = rng.standard_normal(Bsh).astype(np.float32).astype(np.float64)
    C0 = rng.standard_normal((m, n)).astype(np.float32).astype(np.float64)
    opA = (np.tril(A) + np.tril(A, -1).T) if opa == "S" else (A if opa == "N" else A.T)
    opB = B if opb == "N" else B.T
    alpha, beta = 1.0, 0.5
    ref = alpha * (opA @ opB) + beta * C0
    bound = (3 * 2.0 ** -17 + k * 2.0 ** -24) * (np.abs(opA) @ np.abs(opB)) + 2.0 ** -23 * np.abs(ref) + 1e-30
    dC = dev32(C0)
    wb = ctx.evd_sgemm_x3_work_size(m, n, k)
    work = torch.empty(max(wb // 4, 1), dtype=torch.float32, device="cuda")
    ctx.evd_sgemm_x3(opa, opb, lower, m, n, k, alpha, dev32(A), A.shape[0], dev32(B), B.shape[0], beta, dC, m,
                     work, wb)
    torch.cuda.synchronize()
    out = host32(dC, m, n)
    err = np.abs(out - ref)
    if lower:
        mask = np.tril(np.ones((m, n), bool))
        assert np.all(err[mask] <= bound[mask])
        assert np.array_equal(out[~mask], C0[~mask])
    else:
        assert np.all(err <= bound), float((err / bound).max())
    if k >= 1024 and not lower:
        rel = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        assert rel < 2e-5  # split-BF16x3 keeps ~17 bits; plain bf16 would be ~3e-3
