"""Benchmark of the FP64 LU and Cholesky factorizations on one MI355X.

One step = FP64 LU with partial pivoting (dgetrf) of an N x N matrix with
uniform[-1, 1] entries + FP64 Cholesky (dpotrf) of an N x N SPD matrix
B B^T / N + I, both resident in HBM before the timed region (one fresh copy
per step, made before timing).  value = (2N^3/3 + N^3/3) / time, TFLOP/s.

Prints one JSON line (rank 0) with the roofline of the dominant kernel (the
FP64 Schur-complement update GEMM, timed with HIP events on the stream it is
launched on) and the CPU oracle's throughput on a bounded sample.
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
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=32768)
    p.add_argument("--cpu-steps", type=int, default=24, help="elimination steps in the oracle sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-chol", action="store_true")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spd_on_device(n, torch, cdf, workloads):
    """A = B B^T / n + I from the seeded B (input generation on the GPU)."""
    rng = np.random.default_rng(workloads.SEED_MATRIX)
    b = torch.from_numpy(rng.standard_normal(size=(n, n))).cuda()
    s = torch.matmul(b, b.t().contiguous()) / n
    del b
    s.diagonal().add_(1.0)
    s = torch.tril(s) + torch.tril(s, -1).t()
    out = cdf.cm_empty(n, n)
    out.copy_(s)
    del s
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_2108_09337_amd as cdf
    import workloads

    torch.cuda.set_device(0)
    n = args.n
    K, W = args.steps, args.warmup
    h = cdf.handle()
    lu_nb = h.get_param("lu_nb") or 256
    chol_nb = h.get_param("chol_nb") or 128

    log(f"generating inputs n={n}")
    a_host = workloads.lu_uniform(n)
    A0 = cdf.to_device(a_host)
    lu_copies = [A0.clone() for _ in range(K + W)]
    chol_copies = []
    if not args.no_chol:
        S0 = spd_on_device(n, torch, cdf, workloads)
        chol_copies = [S0.clone() for _ in range(K + W)]
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    info_lu = torch.zeros(1, dtype=torch.int32, device="cuda")
    info_ch = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    def step(i, ev=None):
        if ev:
            ev[0].record()
        cdf.dgetrf(lu_copies[i], ipiv, info_lu)
        if ev:
            ev[1].record()
        if chol_copies:
            cdf.dpotrf(chol_copies[i], info_ch)
        if ev:
            ev[2].record()

    for i in range(W):
        log(f"warmup step {i}")
        step(i)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    log(f"timing {K} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        step(W + i, evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert int(info_lu.item()) == 0 and (not chol_copies or int(info_ch.item()) == 0)
    ms = (t1 - t0) * 1e3 / K
    t_lu = np.mean([e[0].elapsed_time(e[1]) for e in evs]) * 1e-3
    t_ch = np.mean([e[1].elapsed_time(e[2]) for e in evs]) * 1e-3
    flops_lu = 2.0 * n ** 3 / 3.0
    flops_ch = n ** 3 / 3.0 if chol_copies else 0.0
    value = (flops_lu + flops_ch) / (ms * 1e-3) / 1e12
    log(f"ms/step {ms:.1f}  LU {flops_lu / t_lu / 1e12:.2f} TF  Chol {flops_ch / max(t_ch, 1e-12) / 1e12:.2f} TF")

    # Dominant kernel: the FP64 Schur-complement update GEMM, replayed with the
    # shapes of one LU's trailing updates on a spent copy, timed with events.
    C = lu_copies[W]
    shapes = []
    for k in range(0, n, lu_nb):
        kb = min(lu_nb, n - k)
        rest = n - k - kb
        if rest > 0:
            shapes.append((k, kb, rest))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for k, kb, rest in shapes:
        cdf.dgemm_update(C[k + kb:, k:k + kb], C[k:k + kb, k + kb:], C[k + kb:, k + kb:])
    e1.record()
    torch.cuda.synchronize()
    gemm_s = e0.elapsed_time(e1) * 1e-3
    gemm_flops = sum(2.0 * rest * rest * kb for _, kb, rest in shapes)
    avg_launch = gemm_s / len(shapes)
    achieved = gemm_flops / len(shapes) / avg_launch / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
                "kernel": "dgemm_kernel (FP64 Schur-complement update, C -= A B)",
                "launches": len(shapes), "avg_launch_us": round(avg_launch * 1e6, 2),
                "flops_per_launch": gemm_flops / len(shapes)}

    cpu = None
    if not args.no_cpu:
        import oracle
        s = args.cpu_steps
        log(f"oracle sample: first {s} elimination steps of the n={n} LU and Cholesky")
        t = time.perf_counter()
        oracle.dgetrf(a_host, ksteps=s)
        t_cl = time.perf_counter() - t
        f = oracle.lu_step_flops(n, s)
        if chol_copies:
            s_host = cdf.to_host(S0)
            t = time.perf_counter()
            oracle.dpotrf(s_host, ksteps=s)
            t_cc = time.perf_counter() - t
            f += oracle.chol_step_flops(n, s)
            t_cl += t_cc
        cpu = {"value": round(f / t_cl / 1e12, 6), "unit": "TFLOP/s", "cores": oracle.get_threads(),
               "kind": "oracle",
               "sample": f"first {s} elimination steps of the n={n} LU (and Cholesky) on the same inputs, "
                         f"{t_cl:.1f} s"}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms, 2), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"FP64 LU (uniform[-1,1]) + FP64 Cholesky (B B^T/N + I), N={n}, one matrix each per step", "n": n, "lu_nb": lu_nb, "chol_nb": chol_nb},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {"lu_tflops": round(flops_lu / t_lu / 1e12, 3),
                   "chol_tflops": round(flops_ch / t_ch / 1e12, 3) if chol_copies else None,
                   "lu_s": round(t_lu, 4), "chol_s": round(t_ch, 4) if chol_copies else None,
                   "frac_fp64_peak": round(value / FP64_PEAK_TFLOPS, 4)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
