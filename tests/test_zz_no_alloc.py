"""The allocation-free evd_dsyevd variant (static device scratch) against
evd_dsyevd with a caller workspace, through the C ABI: same kernels, so the
eigenvalues and eigenvectors must agree bit for bit; both are also held to
the oracle's gates.  Two calls in a row on one context, the second smaller,
so the second finds the first call's contents in the shared scratch."""
import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(ctx, A, jobz, noalloc):
    import torch
    n = A.shape[0]
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()   # column-major
    w = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    if noalloc:
        ctx.evd_dsyevd_noalloc(jobz, "L", n, Ad, n, w, info)
    else:
        wb = ctx.evd_dsyevd_work_size(jobz, "L", n, n)
        work = torch.empty(wb // 8 + 32, dtype=torch.float64, device="cuda")
        ctx.evd_dsyevd(jobz, "L", n, Ad, n, w, work, wb, info)
    torch.cuda.synchronize()
    Q = Ad.cpu().numpy().T if jobz == "V" else None
    return w.cpu().numpy(), Q, int(info.item())


@pytest.mark.parametrize("jobz,sizes", [("V", (1000, 333)), ("N", (5000, 1200))])
def test_noalloc_matches_workspace_entry_point(jobz, sizes):
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    for k, n in enumerate(sizes):
        print(f"noalloc jobz={jobz} call {k} n={n}", flush=True)
        A = W.gaussian_sym(n, seed=600 + n)
        w0, Q0, i0 = _run(ctx, A, jobz, noalloc=False)
        w1, Q1, i1 = _run(ctx, A, jobz, noalloc=True)
        assert i0 == 0 and i1 == 0
        assert np.array_equal(w0, w1)
        if jobz == "V":
            assert np.array_equal(Q0, Q1)
        w_ref = oracle.syev(A, jobz="N")
        assert M.eig_error(w1, w_ref) <= 1e-12
        if jobz == "V":
            assert M.residual(A, w1, Q1) <= 10 and M.orthogonality(Q1) <= 10


def test_noalloc_rejects_sizes_beyond_the_scratch():
    """Host-side check before any launch: n = 2048 with vectors needs more
    than the static scratch."""
    import torch
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    n = 2048
    A = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    w = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(evd.EvdError) as e:
        ctx.evd_dsyevd_noalloc("V", "L", n, A, n, w, info)
    assert e.value.status == evd.EVD_ERR_WORKSPACE
    assert e.value.arg == 4
