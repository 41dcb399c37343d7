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


@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("n,b,mrows", [(40, 2, 40), (100, 4, 77), (300, 16, 300), (333, 32, 129),
                                       (500, 64, 500), (130, 64, 1), (701, 64, 203), (97, 16, 64)])
def test_bcback_matches_generation_order(n, b, mrows, trans):
    """Blocked matrix-core path (b = 16, 32, 64) and reflector-by-reflector
    kernel (other b) against X Q_d / X Q_d^T formed from the reflectors."""
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    B = random_band(n, b, seed=n + b)
    d, e, V, TAU, steps = run_bc(B, b)
    Qb = q_from_reflectors(n, b, V, TAU, steps)
    X = W.rng(5).standard_normal((mrows, n))
    ref = X @ (Qb if trans == "N" else Qb.T)
    dX = to_dev(X)
    dV = to_dev(V.reshape(-1))
    dT = to_dev(TAU.reshape(-1))
    wb = ctx.evd_dbcback_work_size(n, b)
    assert (wb > 0) == (b in (16, 32, 64))
    work = work_dev(wb)
    ctx.evd_dbcback(trans, mrows, n, b, dV, dT, dX, mrows, work, wb)
    torch.cuda.synchronize()
    out = from_dev(dX, mrows, n)
    assert np.max(np.abs(out - ref)) <= 100 * n * M.EPS * np.abs(X).max()


@pytest.mark.parametrize("n,b,mrows", [(333, 32, 129), (500, 64, 300)])
def test_bcback_blocked_matches_valu_kernel(n, b, mrows):
    """The blocked path and the reflector-by-reflector kernel give the same
    product to rounding; a padded leading dimension is honoured."""
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    B = random_band(n, b, seed=7 * n + b)
    d, e, V, TAU, steps = run_bc(B, b)
    X = W.rng(9).standard_normal((mrows + 5, n))
    dV = to_dev(V.reshape(-1))
    dT = to_dev(TAU.reshape(-1))
    wb = ctx.evd_dbcback_work_size(n, b)
    outs = []
    for valu in (0, 1):
        ctx.set_param("bcback_valu", valu)
        try:
            dX = to_dev(X)
            ctx.evd_dbcback("T", mrows, n, b, dV, dT, dX, mrows + 5, work_dev(wb), wb)
            torch.cuda.synchronize()
        finally:
            ctx.set_param("bcback_valu", 0)
        outs.append(from_dev(dX, mrows + 5, n))
    assert np.array_equal(outs[0][mrows:], X[mrows:])  # rows past m_rows untouched
    assert np.max(np.abs(outs[0] - outs[1])) <= 50 * n * M.EPS * np.abs(X).max()


@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("group,rows,sub,rt,lds2", [(32, 0, 0, 0, 0), (64, 64, 0, 0, 0), (64, 128, 0, 0, 0),
                                                    (64, 64, 16, 0, 0), (64, 128, 32, 0, 0), (64, 128, 64, 0, 0),
                                                    (64, 128, 32, 2, 0), (64, 128, 16, 2, 0), (64, 0, 0, 2, 0),
                                                    (64, 64, 0, 0, 1), (64, 64, 64, 0, 0)])
def test_bcback_b64_group_and_row_variants(trans, group, rows, sub, rt, lds2):
    """b = 64: 32- and 64-sweep groups, 64- and 128-row workgroups, 64-sweep
    groups applied whole or as 16- or 32-sweep block reflectors
    ("bcback_sub"), one or two 16-row tiles per wavefront ("bcback_rt"), on a
    size with a ragged last group (n - 2 not a multiple of 64) and partial
    workgroups and row tiles (m_rows not a multiple of 128 or 32); 64-row
    workgroups with one LDS buffer (two per compute unit, the default) or two
    ("bcback_lds2")."""
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    n, b, mrows = 389, 64, 300
    B = random_band(n, b, seed=11)
    d, e, V, TAU, steps = run_bc(B, b)
    Qb = q_from_reflectors(n, b, V, TAU, steps)
    X = W.rng(13).standard_normal((mrows, n))
    ref = X @ (Qb if trans == "N" else Qb.T)
    dX = to_dev(X)
    dV = to_dev(V.reshape(-1))
    dT = to_dev(TAU.reshape(-1))
    wb = ctx.evd_dbcback_work_size(n, b)
    ctx.set_param("bcback_group", group)
    ctx.set_param("bcback_rows", rows)
    ctx.set_param("bcback_sub", sub)
    ctx.set_param("bcback_rt", rt)
    ctx.set_param("bcback_lds2", lds2)
    try:
        ctx.evd_dbcback(trans, mrows, n, b, dV, dT, dX, mrows, work_dev(wb), wb)
        torch.cuda.synchronize()
    finally:
        ctx.set_param("bcback_group", 0)
        ctx.set_param("bcback_rows", 0)
        ctx.set_param("bcback_sub", 0)
        ctx.set_param("bcback_rt", 0)
        ctx.set_param("bcback_lds2", 0)
    out = from_dev(dX, mrows, n)
    assert np.max(np.abs(out - ref)) <= 100 * n * M.EPS * np.abs(X).max()


@pytest.mark.parametrize("case", ["split", "two_rounds", "one_partial_round"])
def test_bcback_b64_automatic_row_split(case):
    """b = 64, automatic workgroup rows: whole rounds of 128-row workgroups
    plus a tail of 64-row ones in a second launch ("split"), a tail too large
    for that ("two_rounds"), and fewer rows than one round of 128-row
    workgroups ("one_partial_round"); every row must match the reflector-by-
    reflector product."""
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    per8, per4 = 128 * cus, 64 * cus
    mrows = {"split": per8 + 100, "two_rounds": per8 + per4 + 100, "one_partial_round": per4 + 50}[case]
    n, b = 389, 64
    B = random_band(n, b, seed=17)
    d, e, V, TAU, steps = run_bc(B, b)
    Qb = q_from_reflectors(n, b, V, TAU, steps)
    X = W.rng(19).standard_normal((mrows, n))
    ref = X @ Qb.T
    dX = to_dev(X)
    wb = ctx.evd_dbcback_work_size(n, b)
    ctx.evd_dbcback("T", mrows, n, b, to_dev(V.reshape(-1)), to_dev(TAU.reshape(-1)), dX, mrows, work_dev(wb), wb)
    torch.cuda.synchronize()
    out = from_dev(dX, mrows, n)
    assert np.max(np.abs(out - ref)) <= 100 * n * M.EPS * np.abs(X).max()
