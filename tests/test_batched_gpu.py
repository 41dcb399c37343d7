"""Batched EVD (evd_dsyevd_batched): every matrix of an uneven batch of
tight-binding Hamiltonians against the oracle; the hipGraph replays agree
bitwise with a direct (uncaptured) run, with eager work between replays."""
import numpy as np
import pytest

import oracle
import oracle.metrics as M
from paper_2511_16174_amd import workloads as W

pytestmark = pytest.mark.gpu


def make_batch(count, seed, lmin, lmax):
    Ls, mats = W.tight_binding_batch(count, seed, lmin, lmax)
    return Ls, mats


def run_batched(ctx, mats, graph=1, streams=4, reps=1, plain=1):
    import torch
    ctx.set_param("batch_graph", graph)
    ctx.set_param("batch_streams", streams)
    ctx.set_param("batch_plain", plain)
    ns = [m.shape[0] for m in mats]
    pristine = [torch.from_numpy(np.ascontiguousarray(m.T)).cuda() for m in mats]  # column-major
    As = [p.clone() for p in pristine]
    Ws = [torch.empty(max(n, 1), dtype=torch.float64, device="cuda") for n in ns]
    info = torch.zeros(len(mats), dtype=torch.int32, device="cuda")
    stamps = torch.zeros(2 * len(mats), dtype=torch.int64, device="cuda")
    wb = ctx.evd_dsyevd_batched_work_size("V", ns, ns)
    work = torch.empty(wb // 8 + 32, dtype=torch.float64, device="cuda")
    outs = []
    for r in range(reps):
        for a, p in zip(As, pristine):
            a.copy_(p)                      # eager work between replays
        torch.cuda.synchronize()
        ctx.set_param("last_hip_error", 0)
        try:
            ctx.evd_dsyevd_batched("V", "L", ns, As, ns, Ws, work, wb, info, stamps)
        finally:
            print("hip error:", ctx.get_param("last_hip_error"), "capture error:", ctx.get_param("capture_error"),
                  "graph used:", ctx.get_param("last_graph_used"))
        torch.cuda.synchronize()
        outs.append(([w[:n].cpu().numpy() for w, n in zip(Ws, ns)],
                     [a.cpu().numpy().T.copy() for a in As], info.cpu().numpy().copy(),
                     stamps.cpu().numpy().copy(), ctx.get_param("last_graph_used")))
    ctx.set_param("batch_graph", 0)
    ctx.set_param("batch_plain", 1)
    return outs


def test_batched_direct_single_stream():
    """One internal stream, no graph: the plainest form of the batched call."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    Ls, mats = make_batch(5, seed=3, lmin=3, lmax=8)
    ws, Qs, info, stamps, used = run_batched(ctx, mats, graph=0, streams=1, reps=1)[0]
    ctx.set_param("batch_streams", 0)
    assert used == 0 and np.all(info == 0)
    for A, w, Q in zip(mats, ws, Qs):
        assert M.eig_error(w, oracle.syev(A, jobz="N")) <= 1e-12
        assert M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10


def test_batched_tight_binding_vs_oracle():
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    Ls, mats = make_batch(14, seed=7, lmin=3, lmax=13)
    mats.append(W.gaussian_sym(5, 1))
    mats.append(np.array([[2.0]]))
    outs = run_batched(ctx, mats, graph=1, reps=1)
    ws, Qs, info, stamps, used = outs[0]
    assert np.all(info == 0)
    for A, w, Q in zip(mats, ws, Qs):
        w_ref = oracle.syev(A, jobz="N")
        assert M.eig_error(w, w_ref) <= 1e-12
        assert M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10
    st = stamps.reshape(-1, 2)
    assert np.all(st[:, 1] >= st[:, 0]) and np.all(st[:, 0] > 0)


def test_batched_graph_replays_match_direct_run():
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    Ls, mats = make_batch(10, seed=11, lmin=4, lmax=12)
    direct = run_batched(ctx, mats, graph=0, reps=1)[0]
    assert direct[4] == 0
    replays = run_batched(ctx, mats, graph=1, reps=3)
    for ws, Qs, info, _, used in replays:
        assert np.all(info == 0)
        for a, b in zip(ws, direct[0]):
            assert np.array_equal(a, b)
        for a, b in zip(Qs, direct[1]):
            assert np.array_equal(a, b)
    print("graph used on replays:", [r[4] for r in replays])


def test_autotune_picks_a_candidate_and_keeps_parity():
    from paper_2511_16174_amd import evd
    import torch
    ctx = evd.context(0)
    n = 700
    A = W.gaussian_sym(n, seed=5)
    dA = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    wb = ctx.evd_autotune_work_size("V", n)
    work = torch.empty(wb // 8 + 32, dtype=torch.float64, device="cuda")
    b, ms = ctx.evd_autotune("V", n, dA, n, work, wb)
    assert b in (16, 32, 64) and ms > 0
    nb, sub = ctx.get_param("last_tuned_nb"), ctx.get_param("last_tuned_sub")
    assert nb in (256, 320, 512)
    assert (sub in (32, 64)) if b == 64 else sub == 0
    w, Q = evd.eigh(dA, jobz="V")
    torch.cuda.synchronize()
    w, Q = w.cpu().numpy(), Q.cpu().numpy()
    assert M.eig_error(w, oracle.syev(A, jobz="N")) <= 1e-12
    assert M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10


def test_batched_nonfinite_matrix_sets_only_its_own_status():
    """One matrix of the batch holds a NaN: its info entry reports
    EVD_ERR_NONFINITE and NaN outputs; every other matrix is solved."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    Ls, mats = make_batch(6, seed=13, lmin=4, lmax=10)
    bad = 3
    mats[bad] = mats[bad].copy()
    mats[bad][2, 2] = np.nan
    ws, Qs, info, _, used = run_batched(ctx, mats, graph=1, reps=1)[0]
    assert info[bad] == evd.EVD_ERR_NONFINITE
    assert np.all(np.isnan(ws[bad])) and np.all(np.isnan(Qs[bad]))
    for i, (A, w, Q) in enumerate(zip(mats, ws, Qs)):
        if i == bad:
            continue
        assert info[i] == 0
        assert M.eig_error(w, oracle.syev(A, jobz="N")) <= 1e-12
        assert M.residual(A, w, Q) <= 10 and M.orthogonality(Q) <= 10


def test_batched_bj_c5_full_batch():
    """The batched workload at its real size: 256 tight-binding Hamiltonians,
    L ~ U{8..45} (n = 64..2025), on-site energies U[-2, 2], seed 7, with
    vectors, in one captured graph.  rho_res and rho_orth of every matrix
    (torch FP64 products on the GPU); eigenvalues of 8 matrices spread over
    the size range against the CPU oracle; device timestamps ordered."""
    import torch
    from paper_2511_16174_amd import evd
    from tests.gpu_helpers import device_ratios
    ctx = evd.context(0)
    Ls, mats = make_batch(256, seed=7, lmin=8, lmax=45)
    ws, Qs, info, stamps, used = run_batched(ctx, mats, graph=0, streams=8, reps=1)[0]
    ctx.set_param("batch_streams", 0)
    assert np.all(info == 0)
    worst_res = worst_orth = 0.0
    for A, w, Q in zip(mats, ws, Qs):
        assert np.all(np.diff(w) >= 0)
        res, orth = device_ratios(torch.from_numpy(A).cuda(), torch.from_numpy(w).cuda(),
                                  torch.from_numpy(np.ascontiguousarray(Q)).cuda())
        worst_res, worst_orth = max(worst_res, res), max(worst_orth, orth)
    print(f"BJ.c5: worst rho_res={worst_res:.3f} worst rho_orth={worst_orth:.3f} graph={used}")
    assert worst_res <= 10 and worst_orth <= 10
    order = np.argsort([m.shape[0] for m in mats])
    for i in order[np.linspace(0, len(mats) - 1, 8).astype(int)]:
        assert M.eig_error(ws[i], oracle.syev(mats[i], jobz="N")) <= 1e-12, (i, mats[i].shape[0])
    st = stamps.reshape(-1, 2)
    assert np.all(st[:, 1] >= st[:, 0]) and np.all(st[:, 0] > 0)


def test_batched_plain_launches_match_cooperative():
    """The persistent kernels launched plainly (streams side by side, the
    default) give bit for bit the results of cooperative launches."""
    from paper_2511_16174_amd import evd
    ctx = evd.context(0)
    Ls, mats = make_batch(24, seed=21, lmin=6, lmax=30)
    coop = run_batched(ctx, mats, graph=0, streams=8, reps=1, plain=0)[0]
    plain = run_batched(ctx, mats, graph=0, streams=8, reps=1, plain=1)[0]
    ctx.set_param("batch_streams", 0)
    assert np.all(coop[2] == 0) and np.all(plain[2] == 0)
    for a, b in zip(coop[0], plain[0]):
        assert np.array_equal(a, b)
    for a, b in zip(coop[1], plain[1]):
        assert np.array_equal(a, b)
    for i in (0, len(mats) // 2, len(mats) - 1):
        A = mats[i]
        assert M.eig_error(plain[0][i], oracle.syev(A, jobz="N")) <= 1e-12
        assert M.residual(A, plain[0][i], plain[1][i]) <= 10 and M.orthogonality(plain[1][i]) <= 10
