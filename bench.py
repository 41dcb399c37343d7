"""Benchmark: plain FP64 dense symmetric EVD with eigenvectors on one MI355X.

One step = one full evd_dsyevd call (SBR, BC, D&C, SBR-back, BC-back, final
GEMM) on an n x n matrix that is already resident in HBM; the matrix is
restored from a device copy before each call (the copy is inside the timed
region and costs well under 1% of a step).

Workload: n = 32768, A = (G + G^T) / (2 sqrt(n)), G iid N(0, 1) drawn on the
GPU from torch's Philox generator seeded with 3; band width b = 64.
Metric: EVD TFLOPS at the 4n^3/3 convention (T3 = (4n^3/3)/t), plus time to
solution; T1 = 4n^3/t (the paper's convention) is reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--b B]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (MFMA and vector)
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel: str, n: int, b: int):
    """HBM bytes per launch of `kernel` at this workload, from the committed
    rocprofv3 counter summary profiles/<kernel>_n<n>_b<b>_traffic.md
    (FETCH_SIZE and WRITE_SIZE runs of this same bench command, each scaled by
    what the counter reads for a plain device copy of known size).  None when
    there is no summary or the kernel's source has changed since the counters
    were taken (the summary records the source file's SHA-256)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_n{n}_b{b}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    try:
        src = os.path.join(ROOT, fields["source"])
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != fields["source_sha256"]:
                return None
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def cpu_baseline(n: int = 3072):
    """The CPU oracle (one-stage Householder + implicit QL, with vectors) on a
    bounded sample of the same workload: one n x n matrix of the same recipe."""
    import numpy as np
    import oracle
    from paper_2511_16174_amd import workloads

    A = workloads.gaussian_sym(n, seed=3, scaled=True)
    t0 = time.perf_counter()
    oracle.syev(A, jobz="V")
    t = time.perf_counter() - t0
    return {
        "value": (4.0 * n ** 3 / 3.0) / t / 1e12,
        "unit": "TFLOPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"one n={n} matrix of the same recipe, eigenvalues+vectors, {t:.2f} s",
        "seconds": t,
        "n": n,
    }


def known_logspaced_gpu(n: int, seed: int, reflectors: int = 64):
    """A = H_1 ... H_64 diag(lam) H_64 ... H_1 with |lam| log-spaced over
    [1e-6, 1] and random signs: the recipe of workloads.known_spectrum
    ('logspaced', 64 reflectors; same PCG64 draws in the same order), with the
    two-sided reflector updates done on the GPU."""
    import numpy as np
    import torch
    from paper_2511_16174_amd import workloads

    r = workloads.rng(seed)
    V = workloads.reflector_vectors(n, reflectors, r)
    lam = workloads.logspaced_spectrum(n, r)
    A = torch.diag(torch.from_numpy(lam).cuda())
    for v in V[::-1]:
        v = torch.from_numpy(v / np.linalg.norm(v)).cuda()
        Av = A @ v
        vAv = float(v @ Av)
        A -= 2.0 * torch.outer(v, Av)
        A -= 2.0 * torch.outer(Av, v)
        A += 4.0 * vAv * torch.outer(v, v)
    A = 0.5 * (A + A.t())
    return A.contiguous(), lam


def known_uniform_inplace(n: int, seed: int, reflectors: int = 64):
    """A = H_1 ... H_64 diag(lam) H_64 ... H_1 with lam uniform on [-1, 1]
    (the recipe of workloads.known_spectrum('uniform'); same PCG64 draws in
    the same order), assembled on the GPU without n x n temporaries (a
    matrix of 77 GB at n = 98304): per reflector p = A v, w = p - (v.p) v,
    then the rank-2 update A -= 2 (v w^T + w v^T) in place."""
    import numpy as np
    import torch
    from paper_2511_16174_amd import workloads

    r = workloads.rng(seed)
    V = workloads.reflector_vectors(n, reflectors, r)
    lam = np.sort(r.uniform(-1.0, 1.0, size=n))
    A = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    A.diagonal().copy_(torch.from_numpy(lam))
    for v in V[::-1]:
        v = torch.from_numpy(v / np.linalg.norm(v)).cuda()
        p = torch.mv(A, v)
        w = p - torch.dot(v, p) * v
        L = torch.stack([v, w], dim=1)
        R = torch.stack([w, v], dim=0)
        A.addmm_(L, R, alpha=-2.0)
    torch.cuda.synchronize()
    return A, lam


def mixed_vs_fp64(n: int = 16384, seed: int = 5, reps: int = 2, max_sweeps: int = 8, target: float = 1e-13):
    """Mixed precision + FP64 refinement against plain FP64 on the mixed
    workload (log-spaced known spectrum, 64 reflectors), both with vectors and
    the default band width: time to solution (1 warm-up, then the mean of
    `reps` calls) and, for each, the scaled residual ||A Q - Q L||_F/(n ||A||_F),
    the orthogonality ||Q^T Q - I||_F / n and the eigenvalue error against the
    known spectrum, computed with torch FP64 products outside the timed calls.
    The mixed call stops its refinement as soon as residual and orthogonality
    reach `target` (its own check, inside the timed call)."""
    import torch
    from paper_2511_16174_amd import evd

    ctx = evd.context(0)
    saved = {k: ctx.get_param(k) for k in ("b", "timing")}
    ctx.set_param("b", 0)
    ctx.set_param("timing", 0)
    log(f"[bench] building the log-spaced known-spectrum matrix n={n} on the GPU")
    A0, lam = known_logspaced_gpu(n, seed)
    lam_t = torch.from_numpy(lam).cuda()
    A = torch.empty_like(A0)
    W = torch.empty(n, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ach = torch.zeros(8, dtype=torch.float64, device="cuda")
    wb = max(ctx.evd_dsyevd_work_size("V", "L", n, n), ctx.evd_dsyevd_mixed_work_size("V", "L", n, n))
    work = torch.empty(wb // 8 + 64, dtype=torch.float64, device="cuda")
    nA = torch.linalg.norm(A0).item()

    def accuracy():
        Q = A.t()
        res = (torch.linalg.norm(A0 @ Q - Q * W[None, :]) / (n * nA)).item()
        O = Q.t() @ Q
        O.diagonal().sub_(1.0)
        orth = (torch.linalg.norm(O) / n).item()
        eta = (torch.max(torch.abs(W - lam_t)) / torch.max(torch.abs(lam_t))).item()
        return {"scaled_residual": res, "scaled_orth": orth, "eig_error": eta,
                "meets_1e-13": bool(res <= target and orth <= target and eta <= 1e-12)}

    def timed(fn):
        ts = []
        for r in range(reps + 1):
            A.copy_(A0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if r > 0:
                ts.append(time.perf_counter() - t0)
        return sum(ts) / len(ts)

    out = {}
    t = timed(lambda: ctx.evd_dsyevd("V", "L", n, A, n, W, work, wb, info))
    out["fp64"] = {"seconds": round(t, 4), "info": int(info.item()), **accuracy()}
    log(f"[bench] fp64 n={n} {out['fp64']}")
    ctx.set_param("timing", 1)
    t = timed(lambda: ctx.evd_dsyevd_mixed("V", "L", n, A, n, W, max_sweeps, target, work, wb, info, ach))
    names = ["sbr", "bc", "dc", "sbr_back", "bc_back", "final_product", "refinement", "total"]
    mst = {k: round(v, 1) for k, v in zip(names, ctx.stage_times())}
    ctx.set_param("timing", 0)
    a = ach.cpu().tolist()
    out["mixed"] = {"seconds": round(t, 4), "info": int(info.item()), "sweeps": int(a[2]), "stage_ms": mst,
                    "reported_residual": a[0], "reported_orth": a[1], "largest_cluster_last_sweep": int(a[5]),
                    **accuracy()}
    log(f"[bench] mixed n={n} {out['mixed']}")
    out["speedup_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 3)
    out["workload"] = (f"known spectrum, |lam| log-spaced over [1e-6, 1] with random signs, Q from 64 Householder "
                       f"reflectors, n={n}, seed={seed}; target residual and orthogonality {target}")
    del work, A, A0
    for k, v in saved.items():
        ctx.set_param(k, v)
    return out


def mixed_main(args):
    """Only the mixed-vs-FP64 comparison (log-spaced known spectrum, seed 5 at
    n = 16384, 6 at 32768), as one JSON line."""
    n = args.n
    seed = 5 if n == 16384 else 6
    cmp_ = mixed_vs_fp64(n, seed)
    out = {
        "metric": "time-to-solution, mixed precision + FP64 refinement vs plain FP64 at scaled residual 1e-13",
        "value": cmp_["mixed"]["seconds"],
        "unit": "s",
        "higher_is_better": False,
        "n_gpus": 1,
        "fp64_seconds": cmp_["fp64"]["seconds"],
        "speedup_vs_fp64": cmp_["speedup_vs_fp64"],
        "dtype": "f32 (split-bf16x3) + f64 refinement",
        "data": "synthetic",
        "config": {"workload": cmp_["workload"], "n": n, "seed": seed},
        "runs": cmp_,
    }
    print(json.dumps(out), flush=True)


def batched_main(args):
    """The batched workload: 256 tight-binding Hamiltonians on L x L periodic
    lattices, L ~ U{8..45} (n = 64..2025), hopping -1, on-site energies
    U[-2, 2], seed 7, solved with vectors by evd_dsyevd_batched (one captured
    hipGraph launch per batch).  Per-matrix latency from the device
    timestamps the library writes around each matrix (wall_clock64, 100 MHz):
    p50 / p99 by nearest rank of (end - start) and of (end - first start of
    the batch); aggregate TFLOPS = sum 4 n^3 / 3 over the batch / wall time."""
    import numpy as np
    # independent streams need hardware queues of their own to run side by
    # side: HIP maps a process's streams onto GPU_MAX_HW_QUEUES of them (4 by
    # default); read when the runtime starts, so set before the first HIP call
    os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    import torch
    from paper_2511_16174_amd import evd, workloads

    ctx = evd.context(0)
    ctx.set_param("b", 0)
    ctx.set_param("batch_graph", args.batch_graph)
    ctx.set_param("batch_streams", args.batch_streams)
    ctx.set_param("batch_plain", args.batch_plain)
    Ls, mats = workloads.tight_binding_batch(256, 7, 8, 45)
    ns = [m.shape[0] for m in mats]
    pristine = [torch.from_numpy(np.ascontiguousarray(m.T)).cuda() for m in mats]
    del mats
    As = [p_.clone() for p_ in pristine]
    Ws = [torch.empty(n, dtype=torch.float64, device="cuda") for n in ns]
    info = torch.zeros(len(ns), dtype=torch.int32, device="cuda")
    stamps = torch.zeros(2 * len(ns), dtype=torch.int64, device="cuda")
    wb = ctx.evd_dsyevd_batched_work_size("V", ns, ns)
    work = torch.empty(wb // 8 + 32, dtype=torch.float64, device="cuda")
    log(f"[bench] batched: {len(ns)} matrices, n {min(ns)}..{max(ns)}, workspace {wb / 2**30:.2f} GiB")

    def restore():
        for a, p_ in zip(As, pristine):
            a.copy_(p_)
        torch.cuda.synchronize()

    def step():
        ctx.evd_dsyevd_batched("V", "L", ns, As, ns, Ws, work, wb, info, stamps)

    for i in range(args.warmup):
        restore()
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i} graph={ctx.get_param('last_graph_used')}")
    times, lat, lat_launch = [], [], []
    for i in range(args.steps):
        restore()   # inputs back in HBM before the timed call (not timed)
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        st = stamps.cpu().numpy().reshape(-1, 2).astype(np.float64) * 10.0  # 100 MHz ticks -> ns
        lat.extend((st[:, 1] - st[:, 0]) / 1e6)                           # ms
        lat_launch.extend((st[:, 1] - st[:, 0].min()) / 1e6)
        log(f"[bench] step {i} {times[-1] * 1e3:.1f} ms graph={ctx.get_param('last_graph_used')}")
    assert int((info != 0).sum().item()) == 0
    t = sum(times) / len(times)
    flops = sum(4.0 * n ** 3 / 3.0 for n in ns)

    def pct(v, q):
        v = sorted(v)
        return v[max(0, min(len(v) - 1, int(np.ceil(q / 100.0 * len(v))) - 1))]

    # accuracy of the last batch (not timed): torch FP64 products per matrix
    eps = 2.0 ** -52
    worst_res = worst_orth = 0.0
    for a, p_, w in zip(As, pristine, Ws):
        n = w.numel()
        Q = a.t()
        A0 = p_.t()
        worst_res = max(worst_res, (torch.linalg.norm(A0 @ Q - Q * w[None, :]) /
                                    (n * torch.linalg.norm(A0) * eps)).item())
        O = Q.t() @ Q
        O.diagonal().sub_(1.0)
        worst_orth = max(worst_orth, (torch.linalg.norm(O) / (n * eps)).item())
    out = {
        "metric": "batched EVD throughput (sum 4n^3/3 TFLOPS) and per-matrix latency, 256 tight-binding Hamiltonians",
        "value": round(flops / t / 1e12, 4),
        "unit": "TFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 2),
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256 tight-binding Hamiltonians, L x L tori, L ~ U{8..45}, hopping -1, "
                               "on-site U[-2,2], seed 7, with vectors",
                   "batch": len(ns), "n_min": min(ns), "n_max": max(ns), "streams": args.batch_streams,
                   "plain_launches": args.batch_plain, "graph": args.batch_graph,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "latency_ms": {"p50": round(pct(lat, 50), 3), "p99": round(pct(lat, 99), 3),
                       "p50_from_batch_start": round(pct(lat_launch, 50), 3),
                       "p99_from_batch_start": round(pct(lat_launch, 99), 3)},
        "graph_used": ctx.get_param("last_graph_used"),
        "accuracy": {"worst_rho_res": round(worst_res, 3), "worst_rho_orth": round(worst_orth, 3)},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--b", type=int, default=64)
    ap.add_argument("--jobz", default="V")
    ap.add_argument("--matrix", default="gaussian", choices=["gaussian", "known-uniform"],
                    help="known-uniform: lam uniform on [-1, 1] around 64 reflectors, built in place "
                         "(eigenvalue error reported against the known lam)")
    ap.add_argument("--seed", type=int, default=3, help="seed of the known-spectrum matrix")
    ap.add_argument("--order", type=int, default=1,
                    help="0 = reordered stages (Q_s H.. then Q_sb Q_d), 1 = conventional (Q_s (H.. Q_d))")
    ap.add_argument("--bcback-valu", type=int, default=0,
                    help="1 = reflector-by-reflector BC-back on the vector ALUs instead of the blocked MFMA kernel")
    ap.add_argument("--bcback-sub", type=int, default=0, choices=[0, 16, 32, 64],
                    help="sweeps per BC-back block reflector inside a 64-sweep group (0 = library default, 32)")
    ap.add_argument("--bcback-rt", type=int, default=0, choices=[0, 1, 2],
                    help="16-row tiles per wavefront of the 64-sweep BC-back (0 = library default)")
    ap.add_argument("--dc-host", type=int, default=0,
                    help="1 = D&C on the host CPU beside the GPU back transformation (use with --order 0)")
    ap.add_argument("--mode", default="fp64", choices=["fp64", "mixed", "batched"])
    ap.add_argument("--batch-streams", type=int, default=8, help="internal streams of the batched driver")
    ap.add_argument("--batch-graph", type=int, default=0, help="1 = replay the batch as one captured hipGraph")
    ap.add_argument("--hw-queues", type=int, default=16, choices=range(1, 17), metavar="1..16",
                    help="batched mode: hardware queues of the process (GPU_MAX_HW_QUEUES)")
    ap.add_argument("--batch-plain", type=int, default=1,
                    help="1 = the batched driver's persistent kernels use plain (not cooperative) launches")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one plain 1 GiB device copy (the reference kernel for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters of a rocprofv3 --pmc pass)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--overlap-ab", type=int, default=1,
                    help="1 = after the timed steps, time one call with bulge chasing beside SBR (A/B)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision vs FP64 comparison at n = 16384 (run after the timed steps)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)

    if args.copy_calibration:
        import torch
        a = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
        b_ = torch.empty_like(a)
        torch.cuda.synchronize()
        b_.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 1 << 30}), flush=True)
        return

    if args.mode == "mixed":
        mixed_main(args)
        return
    if args.mode == "batched":
        batched_main(args)
        return

    import torch
    from paper_2511_16174_amd import evd

    n, b = args.n, args.b
    dev = torch.device("cuda:0")
    ctx = evd.context(0)
    ctx.set_param("b", b)
    ctx.set_param("timing", 1)
    ctx.set_param("order", args.order)
    ctx.set_param("bcback_valu", args.bcback_valu)
    ctx.set_param("bcback_sub", args.bcback_sub)
    ctx.set_param("bcback_rt", args.bcback_rt)
    ctx.set_param("dc_host", args.dc_host)

    lam_known = None
    if args.matrix == "known-uniform":
        log(f"[bench] building the known-spectrum matrix n={n} in place on the GPU")
        A0, lam_known = known_uniform_inplace(n, seed=args.seed)
    else:
        log(f"[bench] generating n={n} on the GPU")
        g = torch.Generator(device=dev)
        g.manual_seed(3)
        G = torch.randn((n, n), dtype=torch.float64, device=dev, generator=g)
        A0 = (G + G.t()) * (0.5 / n ** 0.5)   # symmetric: row-major == column-major
        del G
    A = torch.empty_like(A0)
    W = torch.empty(n, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    wb = ctx.evd_dsyevd_work_size(args.jobz, "L", n, n)
    work = torch.empty(wb // 8 + 64, dtype=torch.float64, device=dev)
    log(f"[bench] workspace {wb / 2**30:.1f} GiB")

    def step():
        A.copy_(A0)
        ctx.evd_dsyevd(args.jobz, "L", n, A, n, W, work, wb, info)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i} stages(ms)={['%.1f' % x for x in ctx.stage_times()]}")
    stage_sum = [0.0] * 8
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        st = ctx.stage_times()   # the timing mode synchronises on the last stage
        stage_sum = [a + b_ for a, b_ in zip(stage_sum, st)]
        log(f"[bench] step {i} stages(ms)={['%.1f' % x for x in st]}")
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    assert int(info.item()) == 0, "tridiagonal solver did not converge"
    stage_ms = [x / args.steps for x in stage_sum]

    flops3 = 4.0 * n ** 3 / 3.0
    value = flops3 / t / 1e12
    if args.dc_host and args.jobz.upper() == "V":
        names = ["sbr", "bc", "dc_host_cpu", "sbr_back", "bc_back", "wait_copy_final_gemm", "total"]
    elif args.order == 0:
        names = ["sbr", "bc", "dc", "sbr_back", "bc_back", "final_gemm", "total"]
    else:
        names = ["sbr", "bc", "dc", "transpose", "bc_back", "sbr_back_left", "total"]
    stages = {names[i]: round(stage_ms[i], 3) for i in range(7)}

    # roofline of the dominant single-launch kernel, timed live by the
    # per-stage events the library records on its own stream around that one
    # launch: BC-back (2 n^3 FP64 flops per launch) or, in the reordered
    # order, the final GEMM (2 n^3 flops).  Peak: FP64 78.6 TF for both the
    # matrix cores and the vector ALUs (256 CUs x 4 SIMDs x 16 lanes x 2 flops
    # x 2.4 GHz).
    if args.jobz.upper() == "V":
        cand = {"bc_back": stage_ms[4]}
        if args.order == 0 and not args.dc_host:
            cand["final_gemm"] = stage_ms[5]
        kname = max(cand, key=cand.get)
        kms = cand[kname]
        achieved = 2.0 * n ** 3 / (kms * 1e-3) / 1e12
        blocked = args.bcback_valu == 0 and b in (16, 32, 64)
        if kname == "bc_back":
            kdesc = ("bcback_wide_kernel" if b == 64 else "bcback_mfma_kernel") if blocked else "bcback_kernel"
            bound = "mfma" if blocked else "alu"
        else:
            kdesc, bound = "gemm_f64_kernel (final Q_sb Q_d)", "mfma"
        traffic = measured_traffic(kdesc, n, b) if kname == "bc_back" else None
        roofline = {"kernel": kdesc, "bound": bound,
                    "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
                    "algorithmic_flops_per_launch": 2.0 * n ** 3, "launch_ms": round(kms, 3)}
        if traffic:
            roofline["traffic_GBps"] = round(traffic / (kms * 1e-3) / 1e9, 1)
    else:
        roofline = None

    what = "with eigenvectors" if args.jobz.upper() == "V" else "eigenvalues only"
    wl = (f"plain FP64 EVD {what}, n={n}, A=(G+G^T)/(2 sqrt n), G iid N(0,1)" if lam_known is None else
          f"plain FP64 EVD {what}, n={n}, known spectrum: lam uniform on [-1,1], Q from 64 Householder "
          f"reflectors (seed {args.seed})")
    out = {
        "metric": f"EVD TFLOPS (4n^3/3) and time-to-solution, plain FP64 {what}",
        "value": round(value, 4),
        "unit": "TFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 2),
        "time_to_solution_s": round(t, 4),
        "tflops_4n3": round(4.0 * n ** 3 / t / 1e12, 4),
        "frac_fp64_peak": round(value / PEAK_FP64_TFLOPS, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl,
                   "n": n, "b": b, "jobz": args.jobz, "uplo": "L", "seed": 3 if lam_known is None else args.seed,
                   "stage_order": "reordered" if args.order == 0 else "conventional",
                   "dc": "host CPU" if args.dc_host else "GPU"},
        "stage_ms": stages,
        "roofline": roofline,
    }

    if not args.no_verify and args.jobz.upper() == "V":
        # independent check of the timed result (not timed): FP64 GEMMs from torch
        Q = A.t()  # column-major eigenvectors -> Q[i, j] view
        eps = 2.0 ** -52
        with torch.no_grad():
            R = A0 @ Q - Q * W[None, :]
            res = (torch.linalg.norm(R) / (n * torch.linalg.norm(A0) * eps)).item()
            del R
            O = Q.t() @ Q
            O.diagonal().sub_(1.0)
            orth = (torch.linalg.norm(O) / (n * eps)).item()
            del O
            tr = abs(W.sum().item() - torch.trace(A0).item())
        out["accuracy"] = {"rho_res": round(res, 3), "rho_orth": round(orth, 3), "trace_err": tr}

    if lam_known is not None:
        lam_t = torch.from_numpy(lam_known).to(dev)
        out["accuracy_known_spectrum"] = {
            "eig_error": (torch.max(torch.abs(W - lam_t)) / torch.max(torch.abs(lam_t))).item(),
            "trace_err": abs(W.sum().item() - float(lam_known.sum())),
            "ascending": bool((W[1:] >= W[:-1]).all().item())}
        log(f"[bench] known spectrum: {out['accuracy_known_spectrum']}")
    if args.overlap_ab and args.jobz.upper() == "V":
        # A/B: bulge chasing beside SBR (gated by the band columns SBR
        # publishes) against the timed configuration (after SBR); one warm-up
        # and one timed call with the overlap, after the timed steps
        ctx.set_param("bc_overlap", 1)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        st = ctx.stage_times()
        torch.cuda.synchronize()
        t_ov = time.perf_counter() - t0
        ctx.set_param("bc_overlap", 0)
        out["bc_beside_sbr_ab"] = {
            "after_sbr_ms": round(t * 1e3, 2), "after_sbr_sbr_plus_bc_ms": round(stage_ms[0] + stage_ms[1], 2),
            "beside_sbr_ms": round(t_ov * 1e3, 2), "beside_sbr_sbr_plus_bc_ms": round(st[0] + st[1], 2),
            "info": int(info.item())}
        log(f"[bench] bc beside sbr: {out['bc_beside_sbr_ab']}")
    if not args.no_mixed and args.n == 32768:
        # the metric's second half: mixed precision + refinement against plain
        # FP64 at the 1e-13 scaled residual, on the mixed workload (n = 16384)
        del work, A, A0
        torch.cuda.empty_cache()
        out["mixed_vs_fp64"] = mixed_vs_fp64(16384, 5)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
