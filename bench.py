"""Benchmark of the dense LU / Cholesky hot path on one MI355X.

Headline (``value``): one step = FP64 LU with partial pivoting (dgetrf) of an
N x N matrix with uniform[-1, 1] entries + FP64 Cholesky (dpotrf) of an N x N
SPD matrix B B^T / N + I (N = 65536 by default, the largest size of the
workload's size set; inputs drawn on the GPU with seeded generators and
resident in HBM).  Each step factors scratch copies restored from the inputs
before the step; the steps themselves are bracketed by synchronizations and
timed; value = (2N^3/3 + N^3/3) / time in TFLOP/s.

Also reported (``detail``):
  * sizes: one warm LU and Cholesky at N = 8192 and 32768;
  * mixed: time-to-solution of A x = b (diagonally dominant, N = 65536,
    nrhs = 1) with the BF16 / FP16 update + FP64 refinement to an HPL scaled
    residual <= 16, against the FP64 path (FP64 LU + solve + the same
    residual check) on the same matrix, both with their tuned block sizes;
    speedup = FP64 time / mixed time;
  * batched: 4096 LU/Cholesky problems, N log-uniform in [16, 512], one
    graph replay, FP64 and FP32, aggregate TFLOP/s.

``roofline``: the FP64 Schur-complement update GEMM (dgemm_dl_kernel<0, false, 0>,
the dominant kernel): every launch of it inside the first timed LU step is
bracketed by HIP events on the stream it runs on (the library's kernel-timing
hook); achieved = algorithmic flops per launch / average launch duration.
``traffic``: calibrated HBM bytes per launch from the committed rocprofv3 PMC
summary of this benchmark, when it matches this N, block size and kernel
source.  ``cpu_baseline``: the CPU oracle on the first elimination steps of
the same N x N inputs.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LU/Cholesky TFLOP/s vs FP64 MFMA peak; mixed-prec+IR speedup at residual<=16"
FP64_PEAK = 78.6
FP32_PEAK = 157.3


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=65536)
    p.add_argument("--detail-n", type=int, nargs="*", default=[8192, 32768],
                   help="extra sizes measured once each (LU and Cholesky), reported in detail")
    p.add_argument("--mixed-n", type=int, default=65536, help="order of the diagonally dominant mixed LU solve (0 = skip)")
    p.add_argument("--batch", type=int, default=4096)
    p.add_argument("--kernel-n", type=int, default=65536,
                   help="points of the exponential-kernel Cholesky solve (0 = skip)")
    p.add_argument("--cpu-steps", type=int, default=32, help="elimination steps in the oracle sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-parity", action="store_true",
                   help="skip the full-size backward errors (torch FP64 products) after the timed steps")
    p.add_argument("--no-c1", action="store_true", help="skip the N = 1024 latency leg")
    p.add_argument("--no-chol", action="store_true")
    p.add_argument("--no-mixed", action="store_true")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-tune-cache", action="store_true", help="ignore the autotuner cache")
    p.add_argument("--gemm-tile", type=int, default=0, choices=[0, 64, 128],
                   help="tile of the FP64 update GEMM (0 = the library's choice by size)")
    p.add_argument("--lu-leaf-rows", type=int, default=0, choices=[0, 1, 2],
                   help="force the LU panel leaf's rows per thread (counter-collection runs: 2 halves its grid)")
    p.add_argument("--no-kernel-timing", action="store_true",
                   help="skip the per-launch GEMM timing events (counter-collection runs)")
    p.add_argument("--calibrate-bytes", type=int, default=0,
                   help="first run a plain elementwise kernel reading and writing this many bytes (PMC scale)")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PMC_SUMMARY = os.path.join(ROOT, "profiles", "dgemm_nn_lu_fp64_hbm_traffic.md")
GEMM_SOURCE = os.path.join(ROOT, "paper_2108_09337_amd", "csrc", "gemm_f64.hip")


def gemm_source_sha():
    import hashlib
    with open(GEMM_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_per_launch(n, lu_nb):
    """Calibrated HBM bytes per launch of the update GEMM, from the committed
    rocprofv3 PMC summary (FETCH_SIZE and WRITE_SIZE runs of this benchmark),
    or None when there is none for this N / block size or the kernel source
    has changed since the counters were taken."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    vals = {}
    with open(PMC_SUMMARY) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                vals[k.strip("` ")] = v.strip("` ")
    try:
        if int(vals["n"]) != n or int(vals["lu_nb"]) != lu_nb or vals["gemm_source_sha256"] != gemm_source_sha():
            return None
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy(torch, nbytes):
    """A plain elementwise kernel of known traffic (reads and writes nbytes
    each), so that PMC runs of this command carry their own scale for
    FETCH_SIZE / WRITE_SIZE."""
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()


def events(torch, k):
    return [torch.cuda.Event(enable_timing=True) for _ in range(k)]


def fp64_section(args, torch, cdf, workloads, h, tuned):
    """Headline step: FP64 LU of the uniform matrix + FP64 Cholesky of the SPD
    matrix at N = args.n.  Each factorization works on a scratch copy that is
    restored from the resident input before the step, outside the timed
    region; every step is bracketed by synchronizations and timed."""
    n, K, W = args.n, args.steps, args.warmup
    log(f"FP64: generating inputs on the GPU, n={n}")
    S0 = None if args.no_chol else workloads.spd_bbt_torch(n)
    A0 = workloads.lu_uniform_torch(n)
    A = cdf.cm_empty(n, n)
    S = cdf.cm_empty(n, n) if S0 is not None else None
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    info_lu = torch.zeros(1, dtype=torch.int32, device="cuda")
    info_ch = torch.zeros(1, dtype=torch.int32, device="cuda")
    lu_params = tuned(h, "getrf", n)
    ch_params = tuned(h, "potrf", n)
    if args.lu_leaf_rows:
        h.set_param("lu_leaf_rows", args.lu_leaf_rows)
        lu_params = dict(lu_params, lu_leaf_rows=args.lu_leaf_rows)
    torch.cuda.synchronize()

    def restore():
        A.copy_(A0)
        if S is not None:
            S.copy_(S0)
        torch.cuda.synchronize()

    def use(params, other):
        # the two operations share handle parameters (the update GEMM's tile
        # and occupancy): each runs with its own tuned values
        for k in other:
            h.set_param(k, 0)
        for k, v in params.items():
            h.set_param(k, v)

    def step(ev):
        use(lu_params, ch_params)
        ev[0].record()
        cdf.dgetrf(A, ipiv, info_lu)
        ev[1].record()
        if S is not None:
            use(ch_params, lu_params)
            cdf.dpotrf(S, info_ch)
        ev[2].record()

    for i in range(W):
        log(f"warmup step {i}")
        restore()
        step(events(torch, 3))
        assert cdf.device_status(h) == cdf.CDF_OK
    torch.cuda.synchronize()
    evs = [events(torch, 3) for _ in range(K)]
    log(f"timing {K} steps")
    wall = 0.0
    prof_nn = prof_syrk = prof_u12 = {"launches": 0, "total_ms": 0.0, "flops": 0.0}
    for i in range(K):
        restore()
        timed = i == 0 and not args.no_kernel_timing
        if timed:  # HIP events around every update-GEMM launch of the first timed step, on its stream
            cdf.profile_begin(h)
        t0 = time.perf_counter()
        step(evs[i])
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        assert cdf.device_status(h) == cdf.CDF_OK, "LU panel exchange timed out"
        if timed:
            prof_nn = cdf.profile_end("nn", h)
            prof_syrk = cdf.profile_end("syrk", h)
            prof_u12 = cdf.profile_end("u12", h)
    assert int(info_lu.item()) == 0 and (S is None or int(info_ch.item()) == 0)
    ms = wall * 1e3 / K
    t_lu = float(np.mean([e[0].elapsed_time(e[1]) for e in evs])) * 1e-3
    t_ch = float(np.mean([e[1].elapsed_time(e[2]) for e in evs])) * 1e-3
    flops_lu = 2.0 * n ** 3 / 3.0
    flops_ch = n ** 3 / 3.0 if S is not None else 0.0
    value = (flops_lu + flops_ch) / (ms * 1e-3) / 1e12
    log(f"ms/step {ms:.1f}  LU {flops_lu / t_lu / 1e12:.2f} TF  Chol {flops_ch / max(t_ch, 1e-12) / 1e12:.2f} TF")

    use(lu_params, ch_params)  # the LU's values for what follows (the block size below)
    # dominant kernel: the FP64 update GEMM (Schur-complement updates only;
    # the products forming U12 = L11^-1 A12 are filed apart), every launch of
    # it inside the first timed LU step
    lu_nb = h.get_param("lu_nb") or (512 if n >= 16384 else 256)  # the library's default otherwise
    launches = max(prof_nn["launches"], 1)
    avg = prof_nn["total_ms"] * 1e-3 / launches
    fpl = prof_nn["flops"] / launches
    bpl = prof_nn.get("bytes", 0.0) / launches
    achieved = fpl / avg / 1e12 if avg > 0 else None
    traffic = traffic_per_launch(n, lu_nb)
    roofline = {"bound": "mfma", "achieved": None if achieved is None else round(achieved, 3), "peak": FP64_PEAK,
                "unit": "TFLOP/s", "frac": None if achieved is None else round(achieved / FP64_PEAK, 4),
                "traffic": traffic,
                "kernel": "dgemm_dl_kernel<0, false, 0> (FP64 Schur-complement update C -= A B, direct-to-LDS "
                          "operands; dgemm_kernel<0,0,false> where its shape conditions fail)",
                "launches": prof_nn["launches"], "avg_launch_us": round(avg * 1e6, 2),
                "flops_per_launch": round(fpl, 1),
                "algorithmic_bytes_per_launch": round(bpl, 1),
                "traffic_over_algorithmic": None if not traffic or not bpl else round(traffic / bpl, 3),
                "u12_products": {"launches": prof_u12["launches"], "gflop": round(prof_u12["flops"] * 1e-9, 1),
                                 "ms": round(prof_u12["total_ms"], 2),
                                 "note": "L11^-1 and U12 = L11^-1 A12 as matrix products: work beyond the "
                                         "method's 2N^3/3, not counted in achieved"},
                "syrk": {"launches": prof_syrk["launches"],
                         "tflops": round(prof_syrk["flops"] / max(prof_syrk["total_ms"], 1e-9) * 1e-9, 3)}}
    parity = None
    if not args.no_parity:
        from tests import gpu_util
        log("parity: backward errors of the last LU and Cholesky (torch FP64 products)")
        t0 = time.perf_counter()
        ip_host = ipiv.cpu().numpy()
        parity = {"lu_backward_error": round(gpu_util.lu_backward_error_torch(torch, A0, A, ip_host), 5),
                  "method": "||PA-LU||_F/(||A||_F N eps) and ||A-LL^T||_F/(||A||_F N eps), eps=2^-53, by "
                            "torch FP64 matrix products on the GPU (independent of the library's kernels)"}
        if S is not None:
            parity["chol_backward_error"] = round(gpu_util.chol_backward_error_torch(torch, S0, S), 5)
        log(f"parity: {parity} ({time.perf_counter() - t0:.1f} s)")
        assert parity["lu_backward_error"] <= 10.0 and parity.get("chol_backward_error", 0.0) <= 10.0
        torch.cuda.empty_cache()
    out = {"value": value, "ms": ms, "t_lu": t_lu, "t_ch": t_ch, "flops_lu": flops_lu, "flops_ch": flops_ch,
           "roofline": roofline, "lu_nb": lu_nb,
           "chol_nb": ch_params.get("chol_nb") or (512 if n >= 16384 else 128),  # the library's default otherwise
           "params": {"getrf": lu_params, "potrf": ch_params}, "parity": parity,
           "lu_result": A, "ipiv": ipiv.cpu().numpy(), "chol_result": S}
    for k in list(lu_params) + list(ch_params):
        h.set_param(k, 0)
    del A, S
    return out, A0, S0


def size_detail(args, torch, cdf, workloads, h, tuned):
    """One warm LU and one warm Cholesky at each extra size (event-timed)."""
    res = {}
    for n in args.detail_n:
        A0 = workloads.lu_uniform_torch(n)
        S0 = workloads.spd_bbt_torch(n)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        r = {}
        for name, src, op, fl in (("lu", A0, "getrf", 2.0 * n ** 3 / 3), ("chol", S0, "potrf", n ** 3 / 3.0)):
            params = tuned(h, op, n)
            X = cdf.cm_empty(n, n)
            best = None
            for rep in range(2):
                X.copy_(src)
                e0, e1 = events(torch, 2)
                torch.cuda.synchronize()
                e0.record()
                if name == "lu":
                    cdf.dgetrf(X, ipiv, info)
                else:
                    cdf.dpotrf(X, info)
                e1.record()
                torch.cuda.synchronize()
                assert int(info.item()) == 0
                t = e0.elapsed_time(e1) * 1e-3
                best = t if rep == 1 else best
            r[name] = {"seconds": round(best, 5), "tflops": round(fl / best / 1e12, 3),
                       "frac_peak": round(fl / best / 1e12 / FP64_PEAK, 4), "params": params}
            for k in params:
                h.set_param(k, 0)
            del X
        log(f"n={n}: LU {r['lu']['tflops']} TF, Cholesky {r['chol']['tflops']} TF")
        res[str(n)] = r
        del A0, S0
        torch.cuda.empty_cache()
    return res


def mixed_section(args, torch, cdf, workloads, h, tuned):
    n = args.mixed_n
    if n <= 0:  # only the exponential-kernel solve
        return {"kernel_chol": kernel_chol_section(args, torch, cdf, workloads, h, tuned)} if args.kernel_n else {}
    log(f"mixed: generating diagonally dominant n={n}")
    A = workloads.diag_dominant_torch(n)
    b = workloads.rhs_uniform_torch(n)
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    p64 = tuned(h, "getrf", n)
    pmx = tuned(h, "mixed_getrf", n)
    res = {"n": n, "nrhs": 1, "params": {"fp64": p64, "mixed": pmx}}

    def use(params, other):  # the two LUs share some handle parameters
        for k in other:
            h.set_param(k, 0)
        for k, v in params.items():
            h.set_param(k, v)

    for prec in ("fp64", "bf16", "fp16"):
        use(p64, pmx) if prec == "fp64" else use(pmx, p64)
        cdf.dgesv_mixed(prec, A, b, X, info, max_iter=30, h=h)  # warm-up (also allocates the workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = cdf.dgesv_mixed(prec, A, b, X, info, max_iter=30, h=h)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res[prec] = {"seconds": round(t, 4), "iters": r["iters"], "scaled_resid": round(r["scaled_resid"], 4),
                     "converged": r["converged"], "info": int(info.item())}
        log(f"mixed {prec}: {t:.3f} s, iters {r['iters']}, resid {r['scaled_resid']:.3f}")
    for prec in ("bf16", "fp16"):
        res[prec]["speedup_vs_fp64"] = round(res["fp64"]["seconds"] / res[prec]["seconds"], 3)
    # the BF16 solve again with tournament pivoting in the panel leaves
    h.set_param("lu_pivot", 1)
    try:
        cdf.dgesv_mixed("bf16", A, b, X, info, max_iter=30, h=h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = cdf.dgesv_mixed("bf16", A, b, X, info, max_iter=30, h=h)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
    finally:
        h.set_param("lu_pivot", 0)
    res["bf16_tournament"] = {"seconds": round(t, 4), "iters": r["iters"], "scaled_resid": round(r["scaled_resid"], 4),
                              "converged": r["converged"], "info": int(info.item()),
                              "speedup_vs_fp64": round(res["fp64"]["seconds"] / t, 3),
                              "speedup_vs_partial_pivoting": round(res["bf16"]["seconds"] / t, 3)}
    log(f"mixed bf16 tournament: {t:.3f} s, iters {r['iters']}, resid {r['scaled_resid']:.3f}")
    for group in res["params"].values():
        for k in group:
            h.set_param(k, 0)
    del A, X
    torch.cuda.empty_cache()
    if args.kernel_n:
        res["kernel_chol"] = kernel_chol_section(args, torch, cdf, workloads, h, tuned)
    return res


def kernel_chol_section(args, torch, cdf, workloads, h, tuned):
    """FP8 E4M3 (per-tile scaled) Cholesky update + FP64 refinement on the
    exponential-kernel SPD matrix (n points uniform in the unit cube, length
    0.1, nugget 1e-2), 64 FP64 right-hand sides, against the FP64 path."""
    n, nrhs = args.kernel_n, 64
    log(f"mixed: exponential-kernel matrix n={n}, nrhs={nrhs}")
    A = workloads.exp_kernel_matrix_torch(workloads.kernel_points(n))
    B = workloads.rhs_uniform_torch(n, nrhs, seed=workloads.SEED_POINTS_RHS)
    X = torch.empty_like(B)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    res = {"n": n, "nrhs": nrhs, "params": {"fp64": tuned(h, "potrf", n)}}
    for prec in ("fp64", "e4m3", "bf16"):
        if prec == "fp64":  # warm-up (allocates the workspace, the largest of the three layouts)
            cdf.dposv_mixed(prec, A, B, X, info, max_iter=30, h=h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            r = cdf.dposv_mixed(prec, A, B, X, info, max_iter=30, h=h)
        except cdf.CdfError as e:
            r = {"status": e.status, "converged": False, "iters": None, "scaled_resid": float("nan")}
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res[prec] = {"seconds": round(t, 4), "iters": r["iters"], "scaled_resid": r["scaled_resid"],
                     "converged": r["converged"], "status": r["status"], "info": int(info.item()),
                     "method": r.get("method"), "shift": r.get("shift"), "factorizations": r.get("factorizations"),
                     "corrections": r.get("corrections"), "pcg_iterations": r.get("pcg_iterations")}
        log(f"kernel matrix {prec}: {t:.3f} s, converged {r['converged']}, iters {r['iters']}, "
            f"resid {r['scaled_resid']}, info {int(info.item())}, method {r.get('method')}, "
            f"shift {r.get('shift')}, factorizations {r.get('factorizations')}")
    for prec in ("e4m3", "bf16"):
        if res[prec]["converged"]:
            res[prec]["speedup_vs_fp64"] = round(res["fp64"]["seconds"] / res[prec]["seconds"], 3)
    for k in res["params"]["fp64"]:
        h.set_param(k, 0)
    del A, B, X
    torch.cuda.empty_cache()
    return res


def c1_section(args, torch, cdf, workloads, h, n=1024, reps=50):
    """Latency case: dgetrf + dgetrs of one n = 1024 system (A uniform[-1,1]
    seed 0, b uniform[-1,1] seed 1), event-timed, median of `reps` after 5
    warm-ups; A and b restored by device copies outside the timed region.
    Beside it the CPU oracle's full factor + solve (median of 3, all threads,
    and once on one thread), and the parity of the two results."""
    a = workloads.lu_uniform(n, seed=workloads.SEED_MATRIX)
    b = workloads.rhs_uniform(n, 1, seed=workloads.SEED_RHS)[:, 0]
    A0, B0 = cdf.to_device(a), cdf.to_device(b)
    A, B = cdf.cm_empty(n, n), torch.empty_like(B0)
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    times = []
    for rep in range(5 + reps):
        A.copy_(A0)
        B.copy_(B0)
        e0, e1 = events(torch, 2)
        torch.cuda.synchronize()
        e0.record()
        cdf.dgetrf(A, ipiv, info)
        cdf.dgetrs(A, ipiv, B)
        e1.record()
        torch.cuda.synchronize()
        if rep >= 5:
            times.append(e0.elapsed_time(e1) * 1e-3)
    assert cdf.device_status(h) == cdf.CDF_OK and int(info.item()) == 0
    t_gpu = float(np.median(times))
    out = {"n": n, "gpu_seconds_median": round(t_gpu, 7), "reps": reps,
           "gpu_tflops": round(2.0 * n ** 3 / 3 / t_gpu / 1e12, 4)}
    if not args.no_cpu:
        import oracle
        from tests import gpu_util
        tc = []
        for _ in range(3):
            t0 = time.perf_counter()
            lu_or, ip_or, _ = oracle.dgetrf(a)
            x_or = oracle.dgetrs(lu_or, ip_or, b)
            tc.append(time.perf_counter() - t0)
        threads = oracle.get_threads()
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.dgetrs(*oracle.dgetrf(a)[:2], b)
        t1 = time.perf_counter() - t0
        oracle.set_threads(threads)
        lu, ip, x = cdf.to_host(A), ipiv.cpu().numpy(), B.cpu().numpy()
        tol = gpu_util.lu_parity_tolerance(lu_or)
        out.update({"oracle_seconds_median": round(float(np.median(tc)), 4), "oracle_threads": threads,
                    "oracle_seconds_1thread": round(t1, 4),
                    "pivots_equal": bool(np.array_equal(ip, ip_or)),
                    "max_err_over_tol": round(float(np.max(np.abs(lu - lu_or) / tol)), 4),
                    "backward_error": round(oracle.lu_backward_error(a, lu, ip), 4),
                    "hpl_scaled_residual": round(oracle.hpl_scaled_residual(a, x, b), 4)})
        assert out["pivots_equal"] and out["max_err_over_tol"] <= 1.0 and out["backward_error"] <= 10
        assert out["hpl_scaled_residual"] <= 16
    log(f"C1 n={n}: GPU {t_gpu * 1e3:.3f} ms (median of {reps}); {out}")
    return out


def batched_section(args, torch, cdf, workloads, h, tuned):
    count = args.batch
    sizes = workloads.batch_sizes(count)
    kinds = workloads.batch_kinds(count)
    flops = float(sum(2.0 * n ** 3 / 3 if k == 0 else n ** 3 / 3.0 for n, k in zip(sizes.astype(float), kinds)))
    mats = [workloads.batch_problem(i, int(n), int(k)) for i, (n, k) in enumerate(zip(sizes, kinds))]
    offs = np.concatenate([[0], np.cumsum([m.size for m in mats])])
    host = np.concatenate([m.ravel(order="F") for m in mats])
    out = {"count": count, "flops": flops}
    for dtn, dt, tdt, peak in (("f64", cdf.F64, torch.float64, FP64_PEAK), ("f32", cdf.F32, torch.float32, FP32_PEAK)):
        src = torch.from_numpy(host).to(device="cuda", dtype=tdt)
        buf = torch.empty_like(src)
        es = buf.element_size()
        a_ptrs = torch.tensor([buf.data_ptr() + int(o) * es for o in offs[:-1]], dtype=torch.int64, device="cuda")
        ldas = torch.tensor(sizes, dtype=torch.int32, device="cuda")
        nmax = int(sizes.max())
        piv = torch.zeros((count, nmax), dtype=torch.int32, device="cuda")
        p_ptrs = torch.tensor([piv.data_ptr() + i * nmax * 4 for i in range(count)], dtype=torch.int64,
                              device="cuda")
        info = torch.zeros(count, dtype=torch.int32, device="cuda")
        # the plan takes its launch shape from the tuner's cache itself
        plan = cdf.VBatchPlan(sizes, kinds, dt, h, tuned=not args.no_tune_cache)
        params = plan.params
        times = []
        for rep in range(6):
            buf.copy_(src)
            e0, e1 = events(torch, 2)
            e0.record()
            plan.run(a_ptrs, ldas, p_ptrs, info)
            e1.record()
            torch.cuda.synchronize()
            if rep:
                times.append(e0.elapsed_time(e1) * 1e-3)
        assert int(info.abs().sum().item()) == 0
        t = float(np.median(times))
        out[dtn] = {"seconds": round(t, 6), "tflops": round(flops / t / 1e12, 3),
                    "frac_peak": round(flops / t / 1e12 / peak, 4), "params": params}
        log(f"batched {dtn}: {t * 1e3:.3f} ms, {flops / t / 1e12:.2f} TF")
        plan.close()
        del src, buf
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2108_09337_amd as cdf
    import workloads
    from paper_2108_09337_amd import tune

    torch.cuda.set_device(0)
    h = cdf.handle()
    if args.gemm_tile:
        h.set_param("gemm_tile", args.gemm_tile)
    cache = {} if args.no_tune_cache else tune.load_cache()

    def tuned(hh, op, n, dtype="f64"):
        return tune.apply(hh, op, n, dtype, cache) if cache else {}

    if args.calibrate_bytes:
        calibrate_copy(torch, args.calibrate_bytes)
    fp, A0, S0 = fp64_section(args, torch, cdf, workloads, h, tuned)
    detail = {"lu_tflops": round(fp["flops_lu"] / fp["t_lu"] / 1e12, 3),
              "chol_tflops": round(fp["flops_ch"] / fp["t_ch"] / 1e12, 3) if fp["flops_ch"] else None,
              "lu_s": round(fp["t_lu"], 4), "chol_s": round(fp["t_ch"], 4),
              "frac_fp64_peak": round(fp["value"] / FP64_PEAK, 4), "tuned_params": fp["params"]}
    cpu = None
    lu_res, ip_gpu, ch_res = fp.pop("lu_result"), fp.pop("ipiv"), fp.pop("chol_result")
    if not args.no_cpu:
        import oracle
        from tests import gpu_util
        s = args.cpu_steps
        n = args.n
        log(f"oracle sample: first {s} elimination steps of the n={n} LU and Cholesky")
        a_host = cdf.to_host(A0)
        t = time.perf_counter()
        lu_s, ip_s, _ = oracle.dgetrf(a_host, ksteps=s)
        t_cl = time.perf_counter() - t
        del a_host
        # the sample is also a parity check of the timed LU: identical first
        # pivots, and its first columns of L (rows moved by the GPU's later
        # interchanges) and first rows of U within the rounding tolerance
        assert np.array_equal(ip_gpu[:s], ip_s[:s]), "GPU pivots differ from the oracle's"
        perm = gpu_util.perm_from_ipiv(np.concatenate([np.arange(1, s + 1), ip_gpu[s:]]), n)
        tol = gpu_util.lu_partial_tolerance(np.asfortranarray(lu_s[:, :s]), s, n)
        err = np.abs(lu_res[:, :s].cpu().numpy() - lu_s[perm, :s])
        lu_ratio = float(np.max(err / tol[perm]))
        Lk = np.tril(lu_s[:s, :s], -1) + np.eye(s)
        utol = 16 * n * gpu_util.EPS * (np.abs(Lk) @ np.abs(lu_s[:s, s:])) + 1e-300
        u_ratio = float(np.max(np.abs(lu_res[:s, s:].cpu().numpy() - lu_s[:s, s:]) / utol))
        del lu_s, tol, err, utol, Lk
        f = oracle.lu_step_flops(n, s)
        samples = {"lu_first_pivots_equal": s, "lu_first_cols_max_err_over_tol": round(lu_ratio, 4),
                   "u_first_rows_max_err_over_tol": round(u_ratio, 4)}
        assert lu_ratio <= 1.0 and u_ratio <= 1.0
        if S0 is not None:
            s_host = cdf.to_host(S0)
            t = time.perf_counter()
            l_s, _ = oracle.dpotrf(s_host, ksteps=s)
            t_cl += time.perf_counter() - t
            f += oracle.chol_step_flops(n, s)
            del s_host
            Lk = np.tril(l_s[:, :s])
            ltol = 16 * n * gpu_util.EPS * (np.abs(Lk) @ np.abs(Lk[:s, :]).T) / np.abs(np.diag(Lk))[None, :]
            cerr = np.abs(np.tril(ch_res[:, :s].cpu().numpy()) - Lk)
            samples["chol_first_cols_max_err_over_tol"] = round(float(np.max(cerr / (ltol + 1e-300))), 4)
            assert samples["chol_first_cols_max_err_over_tol"] <= 1.0
            del l_s, Lk, ltol, cerr
        fp["parity"] = dict(fp["parity"] or {}, oracle_sample=samples)
        cpu = {"value": round(f / t_cl / 1e12, 6), "unit": "TFLOP/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"first {s} elimination steps of the n={n} LU and Cholesky factorizations of the "
                         f"benchmark's own inputs ({f:.3e} flop in {t_cl:.1f} s)",
               "cpu_model": oracle.cpu_model(), "host_triad_gbs": round(oracle.host_triad_gbs(), 1)}
    del A0, S0, lu_res, ch_res
    torch.cuda.empty_cache()
    detail["parity"] = fp["parity"]
    if not args.no_c1:
        detail["c1"] = c1_section(args, torch, cdf, workloads, h)
    if args.detail_n:
        detail["sizes"] = size_detail(args, torch, cdf, workloads, h, tuned)
    if not args.no_mixed:
        detail["mixed"] = mixed_section(args, torch, cdf, workloads, h, tuned)
    if not args.no_batched:
        detail["batched"] = batched_section(args, torch, cdf, workloads, h, tuned)

    n = args.n
    out = {
        "metric": METRIC, "value": round(fp["value"], 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(fp["ms"], 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"FP64 LU with partial pivoting (uniform[-1,1]) + FP64 Cholesky (B B^T/N + I), "
                               f"N={n}, one matrix each per step (inputs drawn on the GPU)", "n": n,
                   "lu_nb": fp["lu_nb"],
                   "chol_nb": fp["chol_nb"]},
        "roofline": fp["roofline"],
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
