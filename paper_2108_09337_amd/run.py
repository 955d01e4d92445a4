"""Run one operation of libcdnafact on a seeded synthetic workload and print
its time (for profiling and quick checks).

  python -m paper_2108_09337_amd.run getrf --n 32768 --reps 2
  python -m paper_2108_09337_amd.run potrf --n 32768 --chol-nb 512
  python -m paper_2108_09337_amd.run gesv-mixed --n 65536 --prec bf16
  python -m paper_2108_09337_amd.run vbatch --count 4096 --dtype f64

Inputs are drawn on the GPU (uniform[-1, 1] for LU, B B^T / n + I for
Cholesky, the diagonally dominant matrix and uniform right-hand side for the
mixed solves); the batched workload is the seeded size/kind mix.  Block sizes
come from the autotuner cache unless given explicitly.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("op", choices=["getrf", "potrf", "gesv-mixed", "posv-mixed", "vbatch"])
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--prec", default="bf16", choices=["fp64", "bf16", "fp16", "e4m3"])
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--lu-nb", type=int, default=0)
    ap.add_argument("--chol-nb", type=int, default=0)
    ap.add_argument("--mixed-nb", type=int, default=0)
    ap.add_argument("--gemm-wg", type=int, default=0, help="update-GEMM workgroups per CU (3, 4 or 5)")
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_2108_09337_amd as cdf
    import workloads
    from paper_2108_09337_amd import tune

    torch.cuda.set_device(0)
    h = cdf.handle()
    op_key = {"getrf": "getrf", "potrf": "potrf", "gesv-mixed": "mixed_getrf", "posv-mixed": "mixed_getrf"}
    if args.op in op_key:
        tune.apply(h, op_key[args.op], args.n)
    if args.op == "gesv-mixed":
        tune.apply(h, "getrf", args.n)
    for name, v in (("lu_nb", args.lu_nb), ("chol_nb", args.chol_nb), ("mixed_nb", args.mixed_nb),
                    ("gemm_wg_per_cu", args.gemm_wg)):
        if v:
            h.set_param(name, v)
    n = args.n
    if args.op in ("getrf", "potrf"):
        src = workloads.lu_uniform_torch(n) if args.op == "getrf" else workloads.spd_bbt_torch(n)
        A = cdf.cm_empty(n, n)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        fl = 2.0 * n ** 3 / 3 if args.op == "getrf" else n ** 3 / 3.0
        for rep in range(args.reps):
            A.copy_(src)
            torch.cuda.synchronize()
            t = time.perf_counter()
            if args.op == "getrf":
                cdf.dgetrf(A, ipiv, info, h)
            else:
                cdf.dpotrf(A, info, h=h)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            print(f"{args.op} n={n} {dt * 1e3:.1f} ms {fl / dt / 1e12:.2f} TFLOP/s info={int(info.item())}",
                  flush=True)
    elif args.op in ("gesv-mixed", "posv-mixed"):
        if args.op == "gesv-mixed":
            A = workloads.diag_dominant_torch(n)
        else:
            A = workloads.exp_kernel_matrix_torch(workloads.kernel_points(n))
        B = workloads.rhs_uniform_torch(n, args.nrhs)
        X = torch.empty_like(B)
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        fn = cdf.dgesv_mixed if args.op == "gesv-mixed" else cdf.dposv_mixed
        for rep in range(args.reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = fn(args.prec, A, B, X, info, h=h)
            torch.cuda.synchronize()
            print(f"{args.op} n={n} {args.prec} {time.perf_counter() - t:.3f} s {r}", flush=True)
    else:
        sizes = workloads.batch_sizes(args.count)
        kinds = workloads.batch_kinds(args.count)
        dt = cdf.F64 if args.dtype == "f64" else cdf.F32
        tdt = torch.float64 if dt == cdf.F64 else torch.float32
        tune.apply(h, "vbatch", int(sizes.max()), args.dtype)
        mats = [workloads.batch_problem(i, int(m), int(k)) for i, (m, k) in enumerate(zip(sizes, kinds))]
        offs = np.concatenate([[0], np.cumsum([m.size for m in mats])])
        src = torch.from_numpy(np.concatenate([m.ravel(order="F") for m in mats])).to(device="cuda", dtype=tdt)
        buf = torch.empty_like(src)
        es = buf.element_size()
        a_ptrs = torch.tensor([buf.data_ptr() + int(o) * es for o in offs[:-1]], dtype=torch.int64, device="cuda")
        ldas = torch.tensor(sizes, dtype=torch.int32, device="cuda")
        nmax = int(sizes.max())
        piv = torch.zeros((args.count, nmax), dtype=torch.int32, device="cuda")
        p_ptrs = torch.tensor([piv.data_ptr() + i * nmax * 4 for i in range(args.count)], dtype=torch.int64,
                              device="cuda")
        info = torch.zeros(args.count, dtype=torch.int32, device="cuda")
        plan = cdf.VBatchPlan(sizes, kinds, dt, h)
        fl = float(sum(2.0 * m ** 3 / 3 if k == 0 else m ** 3 / 3.0 for m, k in zip(sizes.astype(float), kinds)))
        for rep in range(args.reps):
            buf.copy_(src)
            torch.cuda.synchronize()
            t = time.perf_counter()
            plan.run(a_ptrs, ldas, p_ptrs, info)
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t
            print(f"vbatch {args.dtype} count={args.count} {dt_s * 1e3:.3f} ms {fl / dt_s / 1e12:.2f} TFLOP/s",
                  flush=True)
        plan.close()


if __name__ == "__main__":
    main()
