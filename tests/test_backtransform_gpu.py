"""Stage 4 (SBR-back and BC-back) on the GPU vs plain numpy application of
the same reflectors (generation order)."""
import numpy as np
import pytest

import oracle.metrics as M
from paper_2511_16174_amd import workloads as W
from tests.gpu_helpers import from_dev, to_dev, work_dev, zeros_dev
from tests.test_bc_gpu import q_from_reflectors, random_band, run_bc
from tests.test_sbr_gpu import q_from_panels, run_sbr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,b", [(10, 4), (100, 8), (300, 32), (257, 64)])
def test_orgsb_matches_panel_product(n, b):
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    A = W.gaussian_sym(n, seed=n)
    AB, Aout, T, p = run_sbr(A, b)
    Q_ref = q_from_panels(Aout, T, n, b, p)
    dA = to_dev(Aout)
    dT = to_dev(T.transpose(0, 2, 1).reshape(-1)) if p else zeros_dev(1)
    dQ = zeros_dev(n * n)
    wb = ctx.evd_dorgsb_work_size(n, b)
    work = work_dev(wb)
    ctx.evd_dorgsb(n, b, dA, n, dT, dQ, n, work, wb)
    torch.cuda.synchronize()
    Q = from_dev(dQ, n, n)
    assert np.max(np.abs(Q - Q_ref)) <= 50 * n * M.EPS
    assert M.orthogonality(Q) <= 10


@pytest.mark.parametrize("n,b,mrows", [(40, 2, 40), (100, 4, 77), (300, 16, 300), (333, 32, 129),
                                       (500, 64, 500), (130, 64, 1)])
def test_bcback_matches_generation_order(n, b, mrows):
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    B = random_band(n, b, seed=n + b)
    d, e, V, TAU, steps = run_bc(B, b)
    Qb = q_from_reflectors(n, b, V, TAU, steps)
    X = W.rng(5).standard_normal((mrows, n))
    ref = X @ Qb
    dX = to_dev(X)
    dV = to_dev(V.reshape(-1))
    dT = to_dev(TAU.reshape(-1))
    ctx.evd_dbcback(mrows, n, b, dV, dT, dX, mrows)
    torch.cuda.synchronize()
    out = from_dev(dX, mrows, n)
    assert np.max(np.abs(out - ref)) <= 100 * n * M.EPS * np.abs(X).max()
