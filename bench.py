"""Benchmark: LSRN least-squares solves on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step is one complete LSRN solve (Alg. 1 or 2): Philox G + FP64 MFMA
sketch, QR + Jacobi SVD, rank cutoff and N, LSQR (or Chebyshev) with fused
one-pass sweeps, x = N y, and double-double refinement to reach relative
error 1e-10.  The default workload is the largest single-GPU problem:
dense m = 1000000, n = 4000 (32 GB of FP64 A), sigma log-spaced 1 .. 1e-8,
b = A x + 1e-6 N(0,1), gamma = 2, tolerance 1e-14 (synthetic, seeded; built
on the GPU before timing).  The precision form (BF16x3 sketch, FP32
sweeps, FP64 refinement) is timed beside it on the same A and b.  Other
workloads: --workload rankdef_200000x2000 (rank 1800) and its transpose,
sparse_2000000x20000, --batch N, --serve.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_MFMA_PEAK_TFS = 78.6    # MI355X dense FP64 matrix
BF16_MFMA_PEAK_TFS = 2500.0  # MI355X dense BF16 matrix
FP64_VECTOR_PEAK_TFS = 78.6  # MI355X FP64 vector: 256 CUs x 64 FMA/clk x 2 x 2.4 GHz

# HBM bytes per launch of a workload's dominant kernel, from rocprofv3
# FETCH_SIZE and WRITE_SIZE passes over this script (averaged over every
# launch of the kernel in one timed solve, like `achieved`), scaled by the
# counters of a plain 1 GiB device copy (FETCH_SIZE reads half the copied
# bytes, WRITE_SIZE all of them).  Commands and per-kernel figures:
# profiles/pmc_sketches.md (the 1e6 x 4000 sketches, counted on
# `--sketch-probe`: the same kernel at the same shape).  An entry is dropped
# when its kernel changes.
MEASURED_TRAFFIC = {
    ("dense_1000000x4000", "fp64", "f64", "sketch_mfma_f64"): 362.6e9,
    ("dense_1000000x4000_k1e6", "fp64", "f64", "sketch_mfma_f64"): 362.6e9,
    ("dense_1000000x4000", "mixed", "f64", "sketch_mfma_bf16x3"): 780.1e9,
    ("dense_1000000x4000_k1e6", "mixed", "f64", "sketch_mfma_bf16x3"): 780.1e9,
}

WORKLOADS = {
    "rankdef_200000x2000": dict(m=200_000, n=2000, rank=1800, smin=1e-6, seed=12, fat=False),
    "rankdef_2000x200000": dict(m=200_000, n=2000, rank=1800, smin=1e-6, seed=112, fat=True),
    "dense_2000x100": dict(m=2000, n=100, rank=100, smin=1e-6, seed=11, fat=False, noise=1e-3),
    # the precision-form workload: full rank, sigma 1 .. 1e-8, b = A x + 1e-6 noise
    "dense_1000000x4000": dict(m=1_000_000, n=4000, rank=4000, smin=1e-8, seed=14, fat=False,
                               noise=1e-6, refine=1, refine_tol=1e-8),
    # the same shape at kappa = 1e6, where kappa u32 < 1 lets the precision form
    # reach the FP64 solution
    "dense_1000000x4000_k1e6": dict(m=1_000_000, n=4000, rank=4000, smin=1e-6, seed=14, fat=False,
                                    noise=1e-6),
}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f, c = math.floor(k), math.ceil(k)
    return xs[f] if f == c else xs[f] + (xs[c] - xs[f]) * (k - f)


def cpu_baseline(T_dev, b_dev, s, d, r, iters_per_solve, sweeps, tall, sample_bytes=1 << 30):
    """The oracle as it stands, timed on a bounded sample of the same solve and
    scaled to solves/s.  T_dev is the tall view (K x d, row-major: A, or the
    array of A^T for an under-determined A).  The sample is the first K' rows
    of T (about 1 GiB); sketch and iteration times grow linearly in K and are
    scaled by K / K'; the QR and one Jacobi sweep of reduced order are scaled
    by their flop counts (d^3 and the solve's sweep count for the Jacobi)."""
    import numpy as np

    import oracle

    t_start = time.perf_counter()
    threads = oracle.num_threads()
    K = T_dev.shape[0]
    Ks = int(min(K, max(d, sample_bytes // (8 * d))))
    T = T_dev[:Ks].cpu().numpy()
    if tall:
        M, b_np = oracle.Matrix.dense(T), b_dev[:Ks].cpu().numpy()
    else:
        M, b_np = oracle.Matrix.dense_colmajor(T), b_dev.cpu().numpy()
    scale_k = K / Ks
    # 1) sketch: the first `rows` rows of G times the sample (each row costs the same)
    rows = max(2, threads)
    t0 = time.perf_counter()
    oracle.sketch(M, rows, 0)
    t_sketch = (time.perf_counter() - t0) * s / rows * scale_k
    # 2) QR of an (s' x d') Gaussian with the same aspect, scaled by flops
    rng = np.random.default_rng(0)
    dq = min(d, 1000)
    sq = int(round(dq * s / d))
    Xq = rng.standard_normal((sq, dq))
    t0 = time.perf_counter()
    Rq = oracle.qr_r(Xq)
    tq = time.perf_counter() - t0
    flops = lambda ss, dd: 2.0 * ss * dd * dd - 2.0 * dd ** 3 / 3.0
    t_qr = tq * flops(s, d) / flops(sq, dq)
    # 3) one Jacobi sweep of order d', scaled by d^3 and the sweep count
    t0 = time.perf_counter()
    oracle.jacobi_rt(Rq, max_sweeps=1)
    t_jac = (time.perf_counter() - t0) * (d / dq) ** 3 * max(1, sweeps)
    # 4) two LSQR iterations on the sample with a preconditioner of the
    #    right shape (the iteration's cost does not depend on its values)
    P = rng.standard_normal((d, r)) / math.sqrt(d)
    t0 = time.perf_counter()
    oracle.lsrn_iterate(M, b_np, P, s, max_iter=2, tol=1e-300)
    # the sample makes 5 products with A or A^T (start: A^T b; each iteration:
    # A v and A^T u); an iteration costs 2
    t_it = (time.perf_counter() - t0) * 2.0 / 5.0 * iters_per_solve * scale_k
    total = t_sketch + t_qr + t_jac + t_it
    return {
        "value": 1.0 / total,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle stages timed on samples and scaled: the first {Ks} of {K} rows of "
                   f"the tall view (x{scale_k:.1f}); sketch of {rows} of {s} rows of G on them "
                   f"(x{s / rows:.0f}); Householder QR of a {sq}x{dq} Gaussian (x flops); one "
                   f"Jacobi sweep of order {dq} (x (d/{dq})^3 x {sweeps} sweeps); LSQR start + 2 "
                   f"iterations on the sample (x 2/5 x {iters_per_solve})"),
        "stage_s": {"sketch": t_sketch, "qr": t_qr, "jacobi": t_jac, "iterations": t_it},
        "sample_wall_s": time.perf_counter() - t_start,
    }


def serve_main(args):
    """The serving workload: Poisson arrivals of uneven dense solves, admitted
    by device-memory footprint onto a pool of streams; reports solves/s and
    latency percentiles.  Each request's A is built on the GPU when it
    arrives (the generator's time is reported, not counted in latency)."""
    import threading

    import numpy as np
    import torch

    import workloads
    from paper_1109_5981_amd import lsrn

    rng = np.random.default_rng(2024)
    nreq, rate = args.serve_requests, args.serve_rate
    dev = torch.device("cuda:0")
    results, lock = {}, threading.Lock()
    srv = lsrn.Server(hbm_budget_bytes=int(args.serve_budget_gb * (1 << 30)),
                      streams=args.serve_streams)
    queue = []           # (ticket, meta, tensors) in submission order
    cv = threading.Condition()
    done_flag = [False]

    def waiter():
        while True:
            with cv:
                while not queue and not done_flag[0]:
                    cv.wait()
                if not queue:
                    return
                ticket, meta, tens = queue.pop(0)
                cv.notify_all()
            x, info, tm = srv.wait(ticket, allow_not_converged=True)
            A, b = tens
            check = None
            if meta["i"] % 16 == 0:
                # accuracy sample: relative normal-equation residual (tall) or
                # relative residual of the consistent system (fat)
                with torch.no_grad():
                    if meta["fat"]:
                        r = b - A.T @ x
                        check = (torch.linalg.norm(r) / torch.linalg.norm(b)).item()
                    else:
                        r = b - A @ x
                        check = (torch.linalg.norm(A.T @ r) /
                                 (torch.linalg.norm(A) * torch.linalg.norm(r))).item()
            with lock:
                results[meta["i"]] = dict(meta, latency_ms=tm["latency_ms"], queue_ms=tm["queue_ms"],
                                          run_ms=tm["run_ms"], status=info["status"],
                                          batch_size=tm["batch_size"],
                                          iters=info["iters"], check=check,
                                          fp64_steps=info.get("fp64_refine_steps", 0))

    # a pool of matrices drawn from the workload's distribution, built before
    # the clock starts; each request takes one at random with a fresh b
    g0 = time.perf_counter()
    pool = []
    for j in range(args.serve_pool):
        while True:
            n = int(rng.integers(16, 513))
            m = int(rng.integers(1000, 100_001))
            if m >= 20 * n:
                break
        cond = 10.0 ** rng.uniform(2, 8)
        pool.append((m, n, cond, workloads.reflected_problem_device(m, n, cond, seed=10_000 + j,
                                                                    device=dev)))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - g0
    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    t_next = t0
    for i in range(nreq):
        t_next += rng.exponential(1.0 / rate)
        m, n, cond, A = pool[int(rng.integers(0, len(pool)))]
        fat = rng.random() < 0.25
        tol = 10.0 ** rng.uniform(-14, -8)
        # half the requests ask for FP32 arithmetic: the precision form serves
        # them where kappa 2^-24 << 1 (cond <= 1e6, over-determined), FP64 otherwise
        fp32 = rng.random() < 0.5
        prec = "mixed" if (fp32 and not fat and cond <= 1e6) else "fp64"
        b = workloads.rhs_gauss_device(n if fat else m, 10_000 + i, device=dev)
        torch.cuda.current_stream().synchronize()   # not the device: solves are running
        now = time.perf_counter()
        if now < t_next:
            time.sleep(t_next - now)
        with cv:
            while len(queue) > args.serve_streams * 8:   # back-pressure on the inputs held
                cv.wait(0.01)
        # method: LSQR for the precision form, Chebyshev for a quarter of the rest
        meth = "chebyshev" if (prec == "fp64" and rng.random() < 0.25) else "lsqr"
        opts = dict(tol=tol, method=meth, precision=prec, seed=i, refine=2 if tol < 1e-12 else 0)
        ticket = srv.submit_dense(A, b, layout=lsrn.COL_MAJOR if fat else lsrn.ROW_MAJOR, **opts)
        with cv:
            queue.append((ticket, dict(i=i, m=n if fat else m, n=m if fat else n, fat=fat,
                                       cond=cond, tol=tol, precision=prec, method=meth), (A, b)))
            cv.notify()
    with cv:
        done_flag[0] = True
        cv.notify()
    th.join()
    t1 = time.perf_counter()
    srv.close()
    lat = [r["latency_ms"] for r in results.values()]
    checks = [r["check"] for r in results.values() if r["check"] is not None]
    status, worst = {}, {}
    for r in results.values():
        key = f'{r["status"]}/{r["precision"]}/{"fat" if r["fat"] else "tall"}/{r["method"]}'
        status[key] = status.get(key, 0) + 1
        if r["check"] is not None and r["check"] >= worst.get(key, {}).get("check", -1.0):
            # the stopping rules bound the preconditioned residual: for
            # under-determined requests the residual of A x = b can be
            # kappa(A) times tol
            worst[key] = {"check": r["check"], "cond": r["cond"], "tol": r["tol"]}
    routes = {}
    for name, sel in (("batched", lambda r: r["batch_size"] > 0), ("single", lambda r: r["batch_size"] == 0)):
        rs = [r for r in results.values() if sel(r)]
        if rs:
            routes[name] = {"count": len(rs),
                            "mean_batch_size": round(float(np.mean([r["batch_size"] for r in rs])), 2),
                            "p50_latency_ms": round(percentile([r["latency_ms"] for r in rs], 50), 3),
                            "mean_run_ms": round(float(np.mean([r["run_ms"] for r in rs])), 3),
                            "mean_queue_ms": round(float(np.mean([r["queue_ms"] for r in rs])), 3)}
    line = {
        "metric": "serving: LS solves/s with p50/p99 latency (Poisson arrivals, uneven shapes)",
        "value": round(len(results) / (t1 - t0), 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64 + precision form",
        "data": "synthetic (seeded; a pool of matrices A = H1..H4 [Sigma V^T; 0], V Haar, sigma "
                "log-spaced to 1/cond, shapes and cond from the workload's distribution; each "
                "request draws one and a fresh b ~ N(0,1))",
        "config": {"workload": "serving_uneven", "requests": nreq, "arrival_rate_per_s": rate,
                   "m": [1000, 100000], "n": [16, 512], "fat_fraction": 0.25,
                   "streams": args.serve_streams, "budget_gb": args.serve_budget_gb,
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "latency_ms": {"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3),
                       "mean_queue": round(float(np.mean([r["queue_ms"] for r in results.values()])), 3)},
        "routes": routes,
        "wall_s": round(t1 - t0, 3),
        "pool_build_s": round(t_gen, 3),
        "pool_size": args.serve_pool,
        "status_counts": {str(k): v for k, v in status.items()},
        "accuracy_sample": {"count": len(checks), "max": max(checks) if checks else None,
                            "median": float(np.median(checks)) if checks else None,
                            "max_by_category": worst},
        "precision_form_fp64_fallbacks": sum(1 for r in results.values() if r["fp64_steps"] > 0),
        # precision-form requests the batcher took: the batched path computes in FP64
        "precision_form_batched_in_fp64": sum(1 for r in results.values()
                                              if r["precision"] == "mixed" and r["batch_size"] > 0),
    }
    print(json.dumps(line))


def sparse_main(args):
    """The sparse workloads.  sparse_2000000x20000: CSR A (2e6 x 2e4, 20
    uniform nonzeros per row plus 10 dense columns at 10% fill, N(0,1)
    values), Tikhonov lambda = 1e-3, LSQR to 1e-12 with one refinement step.
    tnimg_1024x4000000: the under-determined 1024 x 4e6 stand-in for the
    paper's tnimg_4 (about 21 nonzeros per column, DCT-like skew of the rows;
    workloads.tnimg_like), LSQR or Chebyshev (--method) to 1e-14 (Alg. 2)."""
    import numpy as np
    import torch

    import workloads
    from paper_1109_5981_amd import lsrn

    dev = torch.device("cuda:0")
    g0 = time.perf_counter()
    if args.workload == "tnimg_1024x4000000":
        wl = dict(seed=16, lam=0.0)
        S = workloads.tnimg_like(4_000_000, seed=wl["seed"])
        tol, refine = 1e-14, 0
        data = ("synthetic tnimg stand-in (seeded; 1024 DCT-frequency rows, 20 or 21 nonzeros "
                "per column: the DC row always, the others drawn with weight (1+u+v)^-1.5, values "
                "N(0,1) 8/(1+u+v); b ~ N(0,1))")
    else:
        wl = workloads.WORKLOADS["sparse_2000000x20000"]
        S = workloads.sparse_problem(wl["m"], wl["n"], wl["per_row"], wl["n_dense"], wl["fill"],
                                     seed=wl["seed"])
        tol, refine = 1e-12, 1
        data = ("synthetic (seeded CSR: 20 uniform columns per row + 10 dense columns at 10% "
                "fill, N(0,1) values; b ~ N(0,1))")
    A = lsrn.Csr.from_host(S.m, S.n, S.rowptr, S.colind, S.val, device=dev)
    b = workloads.rhs_gauss_device(S.m, wl["seed"], device=dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - g0
    lam = wl["lam"]
    opts = dict(lam=lam, tol=tol, seed=5, refine=refine, method=args.method,
                profile=0 if args.no_profile else 1)
    for _ in range(args.warmup):
        x, info = lsrn.solve_csr(A, b, **opts)
    torch.cuda.synchronize()
    lat, infos = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        x, info = lsrn.solve_csr(A, b, **opts)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        infos.append(info)
    elapsed = time.perf_counter() - t0
    # relative normal-equation residual of the augmented problem [A; lam I]
    # (tall), relative residual of the consistent system (fat)
    Ad = torch.sparse_csr_tensor(A.rowptr, A.colind.long(), A.val, size=(S.m, S.n))
    r = b - Ad @ x
    if S.m >= S.n:
        h = Ad.t().to_sparse_csr() @ r - lam * lam * x
        ne = (torch.linalg.norm(h) / (torch.linalg.norm(A.val) * torch.linalg.norm(r))).item()
    else:
        ne = (torch.linalg.norm(r) / torch.linalg.norm(b)).item()
    info = infos[-1]
    s, d, nnz = info["s"], info["d"], S.nnz
    K = max(S.m, S.n)
    mean = lambda key: sum(i[key] for i in infos) / len(infos)
    kernels = {}
    t_sk = mean("t_sketch_kernel_ms")
    if t_sk > 0:
        # 2 s nnz FP64 flop on the vector ALUs, plus s (m + n) normals
        kernels["sketch_csr"] = {
            "avg_ms": t_sk, "launches_per_step": 1, "bound": "alu",
            "achieved": 2.0 * s * nnz / (t_sk * 1e-3) / 1e12, "unit": "TFLOP/s",
            "peak": FP64_VECTOR_PEAK_TFS}
    t_sw, n_sw = mean("t_sweep_kernel_ms"), mean("sweep_kernels")
    if t_sw > 0 and n_sw > 0:
        avg = t_sw / n_sw
        # one read of the CSR arrays and the long vector (the algorithmic minimum)
        b_iter = 12.0 * nnz + 8.0 * (K + 1) + 16.0 * (S.m + S.n)
        kernels["csr_sweep"] = {
            "avg_ms": avg, "launches_per_step": n_sw, "bound": "hbm",
            "achieved": b_iter / (avg * 1e-3) / 1e9, "unit": "GB/s", "peak": HBM_PEAK_GBS}
    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches_per_step"])
        kk = kernels[dom]
        roofline = {"kernel": dom, "bound": kk["bound"], "achieved": round(kk["achieved"], 4),
                    "peak": kk["peak"], "unit": kk["unit"],
                    "frac": round(kk["achieved"] / kk["peak"], 5), "traffic": None}
    line = {
        "metric": ("LS solves/s (sparse, Tikhonov) at rel normal-equation residual 1e-12"
                   if S.m >= S.n else "LS solves/s (sparse, under-determined, min-length)"),
        "value": round(args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": data,
        "config": {"workload": args.workload, "m": S.m, "n": S.n, "nnz": nnz,
                   "lambda": lam, "gamma": 2.0, "tol": tol, "refine": refine, "method": args.method},
        "latency_ms": {"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3)},
        "stages_ms": {k: round(info[k], 3) for k in ("t_sketch_ms", "t_svd_ms", "t_iter_ms",
                                                     "t_refine_ms", "t_total_ms")},
        "iters": info["iters"], "refine_iters": info["refine_iters"], "rank": info["rank"],
        "s": s, "converged": bool(info["converged"]),
        ("rel_normal_residual" if S.m >= S.n else "rel_residual"): ne,
        "cs_fallbacks": info.get("cs_fallbacks", 0),
        "kernels": kernels, "roofline": roofline, "cpu_baseline": None,
        "setup_s": round(t_gen, 2),
    }
    print(json.dumps(line))


def batch_main(args):
    """Many small uneven tall solves: lsrn_solve_batch (shared launches) against
    the same problems solved one call at a time."""
    import numpy as np
    import torch

    import workloads
    from paper_1109_5981_amd import lsrn

    rng = np.random.default_rng(77)
    dev = torch.device("cuda:0")
    As, bs = [], []
    for i in range(args.batch):
        n = int(rng.integers(16, 257))
        m = int(rng.integers(max(20 * n, 1000), 20_001))
        A, _, _, _ = workloads.dense_problem_device(m, n, smin=10.0 ** -rng.uniform(2, 6),
                                                    seed=20_000 + i, device=dev)
        As.append(A)
        bs.append(workloads.rhs_gauss_device(m, 20_000 + i, device=dev))
    torch.cuda.synchronize()
    opts = dict(seed=5, tol=1e-12)
    lsrn.solve_batch(As, bs, allow_not_converged=True, **opts)        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos = lsrn.solve_batch(As, bs, allow_not_converged=True, **opts)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    xs1 = [lsrn.solve_dense(A, b, allow_not_converged=True, **opts)[0] for A, b in zip(As, bs)]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    diff = max((torch.linalg.norm(a - c) / torch.linalg.norm(c)).item() for a, c in zip(xs, xs1))
    # the same batch with two refinement steps (double-double residuals, CG
    # corrections in shared launches), against the single solves refined
    # the same way (the same automatic preconditioner choice)
    ropts = dict(opts, refine=2)
    lsrn.solve_batch(As, bs, allow_not_converged=True, **ropts)       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xr, infos_r = lsrn.solve_batch(As, bs, allow_not_converged=True, **ropts)
    torch.cuda.synchronize()
    t_batch_r = time.perf_counter() - t0
    xr1 = [lsrn.solve_dense(A, b, allow_not_converged=True, **ropts)[0]
           for A, b in zip(As, bs)]
    torch.cuda.synchronize()
    diff_r = max((torch.linalg.norm(a - c) / torch.linalg.norm(c)).item() for a, c in zip(xr, xr1))
    line = {
        "metric": "batched small LS solves/s (one launch per phase for the whole batch)",
        "value": round(args.batch / t_batch, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic (seeded; U, V Haar, sigma log-spaced to 1e-2..1e-6)",
        "config": {"workload": "batch_small_tall", "problems": args.batch, "m": [1000, 20000],
                   "n": [16, 256], "tol": 1e-12},
        "one_call_per_problem_solves_per_s": round(args.batch / t_single, 2),
        "speedup": round(t_single / t_batch, 3),
        "stage_ms": {"sketch_and_svd": round(infos[0]["t_svd_ms"], 3),
                     "batched_iterations": round(infos[0]["t_iter_ms"], 3)},
        "iters_mean": float(np.mean([i["iters"] for i in infos])),
        "max_rel_diff_vs_single": diff,
        "refined": {"refine": 2, "solves_per_s": round(args.batch / t_batch_r, 2),
                    "batched_iterations_ms": round(infos_r[0]["t_iter_ms"], 3),
                    "refine_iters_mean": float(np.mean([i["refine_iters"] for i in infos_r])),
                    "max_rel_diff_vs_single_refined": diff_r},
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision-steps", type=int, default=3,
                    help="timed solves of the precision form beside the FP64 path (0: none)")
    ap.add_argument("--workload", default="dense_1000000x4000",
                    choices=sorted(WORKLOADS) + ["sparse_2000000x20000", "tnimg_1024x4000000"])
    ap.add_argument("--method", default="lsqr", choices=["lsqr", "chebyshev"])
    ap.add_argument("--refine", type=int, default=None,
                    help="refinement steps (default: 2 for the kappa 1e8 workload, where one "
                         "step leaves about 1e-10, else 1)")
    ap.add_argument("--refine-tol", type=float, default=None,
                    help="relative accuracy of each refinement correction (default: the "
                         "workload's, else the library's 1e-6)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--precond", default="auto", choices=["auto", "svd", "qr"])
    ap.add_argument("--storage", default="f64", choices=["f64", "f32"],
                    help="storage of A handed to the library (f32: lsrn_solve_dense_f32 on the "
                         "FP32-rounded matrix, FP64 arithmetic)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in sweep launch shape")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not time individual kernels with HIP events")
    ap.add_argument("--batch", type=int, default=0,
                    help="run N small uneven solves batched and one by one instead")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving workload instead of the single-solve benchmark")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-rate", type=float, default=500.0)
    ap.add_argument("--serve-streams", type=int, default=8)
    ap.add_argument("--serve-budget-gb", type=float, default=96.0)
    ap.add_argument("--serve-pool", type=int, default=128,
                    help="distinct matrices the requests draw from (built before timing)")
    ap.add_argument("--sketch-probe", action="store_true",
                    help="counter runs: one dense sketch (FP64 MFMA, then BF16x3 with --precision "
                         "mixed) of a Gaussian A of the workload's shape, nothing else")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (3 times); "
                         "its FETCH_SIZE / WRITE_SIZE counters calibrate the traffic figures")
    args = ap.parse_args()

    if args.serve:
        # HIP maps streams onto GPU_MAX_HW_QUEUES hardware queues (4 by
        # default); with more worker streams than queues, streams share a
        # queue and their solves serialise.  Set before the runtime starts.
        os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(32, max(4, args.serve_streams))))
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the solver runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1109_5981_amd import lsrn

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.serve:
        serve_main(args)
        return
    if args.batch > 0:
        batch_main(args)
        return
    if args.workload in ("sparse_2000000x20000", "tnimg_1024x4000000"):
        sparse_main(args)
        return
    dev = torch.device("cuda:0")
    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "launches": 3}))
        return
    wl = WORKLOADS[args.workload]
    if args.sketch_probe:
        sketch_probe(args, wl, dev)
        return
    if args.refine is None:
        args.refine = wl.get("refine", 1)
    t_gen = time.perf_counter()
    A, U, sigma, V = workloads.dense_problem_device(wl["m"], wl["n"], wl["rank"], wl["smin"],
                                                    wl["seed"], device=dev)
    del U, V
    if wl["fat"]:
        # under-determined n x m problem stored column-major: the array of the
        # tall generator read as A^T
        m_ls, n_ls, layout = wl["n"], wl["m"], lsrn.COL_MAJOR
    else:
        m_ls, n_ls, layout = wl["m"], wl["n"], lsrn.ROW_MAJOR
    if "noise" in wl:
        b, _ = workloads.rhs_model_device(A, wl["noise"], wl["seed"])
    else:
        b = workloads.rhs_gauss_device(m_ls, wl["seed"], device=dev)
    torch.cuda.empty_cache()  # the library allocates with hipMalloc, outside torch's cache
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen

    # the warmup solve tunes the sweep's launch shape for this key (autotune);
    # the timed solves reuse the recorded shape
    opts = dict(method=args.method, refine=args.refine, seed=2024, tol=1e-14,
                profile=0 if args.no_profile else 1, precision=args.precision,
                precond=args.precond, autotune=0 if args.no_autotune else 1)
    if args.refine_tol is None:
        args.refine_tol = wl.get("refine_tol")
    if args.refine_tol is not None:
        opts["refine_tol"] = args.refine_tol
    solve = lsrn.solve_dense
    A_solve = A
    if args.storage == "f32":
        # the problem becomes the FP32-rounded matrix
        A_solve = A.float()
        del A
        A = None
        torch.cuda.empty_cache()
        solve = lsrn.solve_dense_f32

    def leg(solve_fn, steps, warmup, A_=None, b_=None, **o):
        """warmup untimed solves, then `steps` timed ones between device syncs."""
        A_ = A_solve if A_ is None else A_
        b_ = b if b_ is None else b_
        for _ in range(warmup):
            x, info = solve_fn(A_, b_, layout=layout, allow_not_converged=True, **o)
        torch.cuda.synchronize()
        lat, infos = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            x, info = solve_fn(A_, b_, layout=layout, allow_not_converged=True, **o)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - ts) * 1e3)
            infos.append(info)
        torch.cuda.synchronize()
        return x, infos, lat, time.perf_counter() - t0

    x, infos, lat, elapsed = leg(solve, args.steps, args.warmup, **opts)

    # accuracy: the same problem solved by the FP64 path with refinement run
    # to convergence (untimed); the oracle parity of these sizes is checked by
    # the GPU test suite
    ref_opts = dict(opts, precision="fp64", refine=6, profile=0, seed=7)
    x_ref, _ = solve(A_solve, b, layout=layout, **ref_opts)
    rel_err = lambda xv: (torch.linalg.norm(xv - x_ref) / torch.linalg.norm(x_ref)).item()
    err_main = rel_err(x)
    Av = A_solve
    if layout == lsrn.ROW_MAJOR:
        res = b - workloads.matvec_device(Av, x)
        ne = torch.linalg.norm(workloads.matvec_device(Av, res, trans=True)) / (
            sigma[0] * torch.linalg.norm(res))
    else:
        res = b - workloads.matvec_device(Av, x, trans=True)
        ne = torch.linalg.norm(workloads.matvec_device(Av, res)) / (sigma[0] * torch.linalg.norm(res))
    ne = ne.item()
    del res

    info = infos[-1]
    s, d, r = info["s"], info["d"], info["rank"]
    K = wl["m"]                              # rows of the tall view
    mean = lambda key, inf=None: sum(i[key] for i in (inf or infos)) / len(inf or infos)
    kernels, stages = kernel_figures(args, infos, s, K, d, mean)

    cpu = None
    if not args.no_cpu_baseline and args.storage == "f64":
        iters_total = info["iters"] + info["refine_iters"] + 2 * info["refine_steps"]
        cpu = cpu_baseline(A_solve, b, s, d, r, iters_total, info["sweeps"], not wl["fat"])

    def leg_summary(xv, infs, latv, el, steps, ref, label_args):
        i_ = infs[-1]
        km, _ = kernel_figures(label_args, infs, s, K, d, lambda key: mean(key, infs))
        return {
            "solves_per_s": round(steps / el, 4),
            "latency_ms": {"p50": round(percentile(latv, 50), 3), "p99": round(percentile(latv, 99), 3)},
            "rel_err_vs_fp64_refined": (torch.linalg.norm(xv - ref) / torch.linalg.norm(ref)).item(),
            "converged": bool(i_["converged"]), "iters": i_["iters"],
            "refine_steps": i_["refine_steps"], "refine_iters": i_["refine_iters"],
            "fp64_refine_steps": i_["fp64_refine_steps"],
            "stages_ms": {k: round(mean(k, infs), 3) for k in
                          ("t_sketch_ms", "t_svd_ms", "t_iter_ms", "t_refine_ms", "t_total_ms")},
            "kernels": km,
        }

    # the precision form beside the FP64 path: on the same A and b, and (for
    # the 1e6 x 4000 problem) on the same shape at kappa 1e6, where FP32
    # sweeps can carry the iterations
    prec_form = None
    if (args.precision == "fp64" and args.storage == "f64" and not wl["fat"]
            and args.precision_steps > 0):
        mixed_args = argparse.Namespace(**dict(vars(args), precision="mixed"))
        # the precision form's refinement runs its own steps (up to 10, each
        # correction to the library's 1e-6)
        o_mixed = dict({k: v for k, v in opts.items() if k != "refine_tol"}, precision="mixed",
                       refine=max(args.refine, 10))
        xm, infos_m, lat_m, el_m = leg(solve, args.precision_steps, 1, **o_mixed)
        prec_form = {"same_problem": leg_summary(xm, infos_m, lat_m, el_m, args.precision_steps,
                                                 x_ref, mixed_args),
                     "note": ("BF16x3 sketch on the BF16 matrix cores, LSQR over an FP32 copy of A, "
                              "refinement residuals in double-double from the FP64 A; when the "
                              "sketch's sigma_max / sigma_min_kept times 2^-24 exceeds 1/2 the "
                              "sweeps read the FP64 A from the start (fp64_refine_steps)")}
        del xm
        if args.workload == "dense_1000000x4000":
            del A_solve, A, x_ref, x
            torch.cuda.empty_cache()
            w6 = WORKLOADS["dense_1000000x4000_k1e6"]
            A6, U6, s6, V6 = workloads.dense_problem_device(w6["m"], w6["n"], w6["rank"], w6["smin"],
                                                            w6["seed"], device=dev)
            del U6, V6
            b6, _ = workloads.rhs_model_device(A6, w6["noise"], w6["seed"])
            torch.cuda.empty_cache()
            # kappa 1e6: one FP64 refinement step with the library's 1e-6 corrections
            o64 = dict({k: v for k, v in opts.items() if k != "refine_tol"}, refine=1)
            x64, i64, l64, e64 = leg(solve, args.precision_steps, 1, A_=A6, b_=b6, **o64)
            ref6, _ = solve(A6, b6, layout=layout, **dict(opts, refine=6, profile=0, seed=7))
            xm6, im6, lm6, em6 = leg(solve, args.precision_steps, 1, A_=A6, b_=b6, **o_mixed)
            prec_form["kappa_1e6"] = {
                "workload": "dense_1000000x4000_k1e6",
                "fp64": leg_summary(x64, i64, l64, e64, args.precision_steps, ref6, args),
                "mixed": leg_summary(xm6, im6, lm6, em6, args.precision_steps, ref6, mixed_args),
                "speedup_mixed_over_fp64": round(e64 / em6, 4),
            }
            del A6, b6, x64, xm6, ref6

    roofline = None
    if kernels:
        dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches_per_step"])
        kk = kernels[dom]
        roofline = {"kernel": dom, "bound": kk["bound"], "achieved": round(kk["achieved"], 3),
                    "peak": kk["peak"], "unit": kk["unit"],
                    "frac": round(kk["achieved"] / kk["peak"], 4),
                    "traffic": MEASURED_TRAFFIC.get((args.workload, args.precision, args.storage, dom))}

    value = args.steps / elapsed
    line = {
        "metric": "LS solves/s + p99 latency at rel err 1e-10; sketch GEMM TFLOP/s, iter GB/s",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64" if args.storage == "f64" else "f64 arithmetic on f32-stored A")
                 if args.precision == "fp64" else "bf16 sketch + f32 sweeps + f64",
        "data": ("synthetic (seeded; A = U diag(sigma) V^T with U, V Haar, sigma log-spaced "
                 "1 .. %g%s; %s)" % (wl["smin"],
                                    ", rank %d" % wl["rank"] if wl["rank"] < min(wl["m"], wl["n"]) else "",
                                    "b = A x + %g N(0,1)" % wl["noise"] if "noise" in wl
                                    else "b ~ N(0,1)")),
        "config": {"workload": args.workload, "m": m_ls, "n": n_ls, "rank": wl["rank"],
                   "gamma": 2.0, "tol": 1e-14, "method": args.method, "refine": args.refine,
                   "refine_tol": args.refine_tol if args.refine_tol is not None else 1e-6,
                   "precision": args.precision, "precond": args.precond, "storage": args.storage,
                   "autotune": not args.no_autotune},
        "tuned_shapes": lsrn.tune_export().strip().splitlines(),
        "latency_ms": {"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3)},
        "rel_err_vs_fp64_refined": err_main,
        "rel_normal_residual": ne,
        "sketch_tflops": round(2.0 * s * K * d / (mean("t_sketch_ms") * 1e-3) / 1e12, 3),
        "iter_gbs": stages.get("iter_phase", {}).get("achieved"),
        "iter_phase": stages.get("iter_phase"),
        "svd_stage": stages.get("svd_stage"),
        "stages_ms": {k: round(mean(k), 3) for k in
                      ("t_sketch_ms", "t_svd_ms", "t_iter_ms", "t_refine_ms", "t_total_ms")},
        "iters": info["iters"], "refine_iters": info["refine_iters"], "rank": r, "s": s,
        "jacobi_sweeps": info["sweeps"],
        "refine_steps": info["refine_steps"],
        "converged": bool(info["converged"]),
        "kernels": kernels,
        "roofline": roofline,
        "precision_form": prec_form,
        "cpu_baseline": cpu,
        "setup_s": round(t_gen, 2),
    }
    print(json.dumps(line))


def sketch_probe(args, wl, dev):
    """One sketch of the workload's shape for hardware-counter passes: A is
    Gaussian (the counters depend on the shapes, not the values), filled in
    row blocks of at most 2^28 entries, and no other library routine runs
    (the solve's input generator calls torch's QR)."""
    import torch
    from paper_1109_5981_amd import lsrn
    # the tall generator's array; a fat workload reads it column-major as A^T
    m, n = wl["m"], wl["n"]
    rows, cols = m, n
    g = torch.Generator(device=dev)
    g.manual_seed(wl["seed"])
    A = torch.empty((rows, cols), dtype=torch.float64, device=dev)
    step = max(1, (1 << 28) // cols)
    for r0 in range(0, rows, step):
        r1 = min(rows, r0 + step)
        A[r0:r1].normal_(generator=g)
    layout = lsrn.COL_MAJOR if wl["fat"] else lsrn.ROW_MAJOR
    s = int(math.ceil(2.0 * min(m, n)))
    out = {"probe": "sketch", "workload": args.workload, "s": s}
    fns = [("fp64", lsrn.sketch_dense)]
    if args.precision == "mixed":
        fns.append(("bf16x3", lsrn.sketch_dense_bf16))
    for name, fn in fns:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X = fn(A, s, seed=1, layout=layout)
        torch.cuda.synchronize()
        out[name + "_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        del X
    print(json.dumps(out))


def kernel_figures(args, infos, s, K, d, mean):
    """Per-kernel rates from the library's HIP-event timings (opt.profile),
    with the algorithmic work of each kernel:
      sketch:       2 s K d flop (one launch);
      row sweep:    one read of A (FP64: 8 K d bytes; FP32 copy: 4 K d) plus
                    the long vector (16 K bytes) per pass; only sweeps that
                    made a pass are timed and counted;
      Jacobi round: the SVD's 11 d^3 flop (eq. for the flop count of LSRN)
                    spread over the solve's round launches.
    and the stage figures: the iteration phase's HBM fraction
    B_iter * passes / (t * 8 TB/s), and the preconditioner stage against the
    FP64 peak: (2 s d^2 + 11 d^3) / t_svd for the SVD, or, when the
    certified full-rank path formed N = R^-1, the flops it made (Householder
    QR 2 s d^2 - 2 d^3 / 3 and the triangular inverse d^3 / 3)."""
    f32 = args.precision != "fp64" or args.storage != "f64"
    bytes_per_sweep = (4.0 if f32 else 8.0) * K * d + 16.0 * K
    t_sketch_k = mean("t_sketch_kernel_ms")
    t_sweep_k, n_sweep = mean("t_sweep_kernel_ms"), mean("sweep_kernels")
    t_jac_k, n_jac = mean("t_jacobi_kernel_ms"), mean("jacobi_kernels")
    sketch_flop = 2.0 * s * K * d
    kernels = {}
    if t_sketch_k > 0 and args.precision == "fp64":
        kernels["sketch_mfma_f64"] = {
            "avg_ms": round(t_sketch_k, 4), "launches_per_step": 1, "bound": "mfma",
            "achieved": round(sketch_flop / (t_sketch_k * 1e-3) / 1e12, 3), "unit": "TFLOP/s",
            "peak": FP64_MFMA_PEAK_TFS}
    elif t_sketch_k > 0:
        # three BF16 products (the exact split of fl32(A)) per element of G A
        kernels["sketch_mfma_bf16x3"] = {
            "avg_ms": round(t_sketch_k, 4), "launches_per_step": 1, "bound": "mfma",
            "achieved": round(3 * sketch_flop / (t_sketch_k * 1e-3) / 1e12, 3), "unit": "TFLOP/s",
            "peak": BF16_MFMA_PEAK_TFS}
    if t_sweep_k > 0 and n_sweep > 0:
        avg = t_sweep_k / n_sweep
        kernels["row_sweep"] = {
            "avg_ms": round(avg, 5), "launches_per_step": n_sweep, "bound": "hbm",
            "achieved": round(bytes_per_sweep / (avg * 1e-3) / 1e9, 1), "unit": "GB/s",
            "peak": HBM_PEAK_GBS}
    if t_jac_k > 0 and n_jac > 0:
        avg = t_jac_k / n_jac
        kernels["jacobi_round"] = {
            "avg_ms": round(avg, 5), "launches_per_step": n_jac, "bound": "alu",
            "achieved": round(11.0 * d ** 3 / n_jac / (avg * 1e-3) / 1e12, 4), "unit": "TFLOP/s",
            "peak": FP64_VECTOR_PEAK_TFS,
            "bytes_per_launch_model": 16.0 * d * d}
    stages = {}
    it, t_it = mean("iters"), mean("t_iter_ms")
    if it > 0 and t_it > 0:
        gbs = bytes_per_sweep * it / (t_it * 1e-3) / 1e9
        stages["iter_phase"] = {"bytes_per_iter": bytes_per_sweep, "iters": it,
                                "t_ms": round(t_it, 3), "achieved": round(gbs, 1), "unit": "GB/s",
                                "peak": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4)}
    t_svd = mean("t_svd_ms")
    if t_svd > 0:
        r_inv = mean("precond_used") == 2
        fl = (2.0 * s * d * d - 2.0 * d ** 3 / 3 + d ** 3 / 3) if r_inv else 2.0 * s * d * d + 11.0 * d ** 3
        tf = fl / (t_svd * 1e-3) / 1e12
        stages["svd_stage"] = {"form": "qr + R^-1 (certified full rank)" if r_inv else "qr + jacobi svd",
                               "flop": fl, "t_ms": round(t_svd, 3), "achieved": round(tf, 3),
                               "unit": "TFLOP/s", "peak": FP64_VECTOR_PEAK_TFS,
                               "frac": round(tf / FP64_VECTOR_PEAK_TFS, 4)}
    return kernels, stages


if __name__ == "__main__":
    main()
