"""Autotuner for the block sizes and launch shapes of libcdnafact.

For each operation it times every candidate of a small search space through
the C-ABI (HIP events on the current stream, fresh inputs per timed call,
best of ``reps``) and records the fastest in a JSON cache keyed by
(operation, element type, size bucket).  ``apply`` sets a handle's
parameters from the cache; the batched plan and the benchmark use it.

  python -m paper_2108_09337_amd.tune --op getrf potrf --n 8192 32768
  python -m paper_2108_09337_amd.tune --op vbatch --count 4096

Search spaces (the parameters the paper tunes are the block size v and the
replication depth, Sec. 7.2 and Sec. 8; on one GPU they become the panel
width, the leaf shape, the update GEMM's tile and occupancy, how U12 is
formed, the pivoting of the mixed LU and the batched launch shape):
  getrf        lu_nb {256, 384, 512}, lu_leaf_rows {1, 2}, gemm_wg_per_cu {4, 5},
               gemm_tile {64, 128}, lu_u12 {0 (L11^-1 product), 1 (substitution)}
  potrf        chol_nb {128, 256, 384, 512}, gemm_wg_per_cu {4, 5} (its products are A B^T
               forms, which have no 128 x 128 variant)
  mixed_getrf  mixed_nb {256, 384, 512}, lu_u12 {0, 1},
               lu_pivot {0 (partial), 1 (tournament)} (BF16 update)
  vbatch       vbatch_nb {0 (32 where it fits), 16}, vbatch_wg_per_cu {1, 2}
Spaces of at most 16 points are searched exhaustively; larger ones by
coordinate descent (each parameter in turn over its values with the others
at their current best, two sweeps, every point timed at most once).
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import time

import numpy as np
import torch

import paper_2108_09337_amd as cdf

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(_HERE, "tune_cache.json")

SPACES = {
    "getrf": {"lu_nb": [256, 384, 512], "lu_leaf_rows": [1, 2], "gemm_wg_per_cu": [4, 5], "gemm_tile": [64, 128],
              "lu_u12": [0, 1]},
    "potrf": {"chol_nb": [128, 256, 384, 512], "gemm_wg_per_cu": [4, 5]},
    "mixed_getrf": {"mixed_nb": [256, 384, 512], "lu_u12": [0, 1], "lu_pivot": [0, 1]},
    "vbatch": {"vbatch_nb": [0, 16], "vbatch_wg_per_cu": [1, 2]},
}
EXHAUSTIVE_MAX = 16


def cache_path() -> str:
    return os.environ.get("CDF_TUNE_CACHE", DEFAULT_CACHE)


def load_cache(path: str | None = None) -> dict:
    p = path or cache_path()
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        return json.load(f)


def save_cache(cache: dict, path: str | None = None) -> None:
    p = path or cache_path()
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def bucket(n: int) -> int:
    """Nearest power of two (size bucket of the cache)."""
    return 1 << max(0, int(round(math.log2(max(1, n)))))


def key(op: str, dtype: str, n: int) -> str:
    return f"{op}/{dtype}/{bucket(n)}"


def apply(h: "cdf.Handle", op: str, n: int, dtype: str = "f64", cache: dict | None = None) -> dict:
    """Set h's parameters for `op` from the cache entry of the nearest bucket; returns them."""
    c = load_cache() if cache is None else cache
    entries = {k: v for k, v in c.items() if k.startswith(f"{op}/{dtype}/")}
    if not entries:
        return {}
    best = min(entries, key=lambda k: abs(math.log2(int(k.rsplit("/", 1)[1])) - math.log2(max(1, n))))
    params = entries[best]["params"]
    for name, v in params.items():
        h.set_param(name, int(v))
    return params


def _search(op, evaluate, spaces=None):
    """Minimize evaluate(params) over the op's space (exhaustive if small,
    else coordinate descent); returns the list of (seconds, params) timed."""
    space = (spaces or SPACES)[op]
    names = sorted(space)
    seen = {}

    def ev(params):
        k = tuple(params[n] for n in names)
        if k not in seen:
            seen[k] = evaluate(dict(params))
        return seen[k]

    if math.prod(len(space[n]) for n in names) <= EXHAUSTIVE_MAX:
        for combo in itertools.product(*(space[n] for n in names)):
            ev(dict(zip(names, combo)))
    else:
        best = {n: space[n][0] for n in names}
        for _ in range(2):
            for n in names:
                ts = []
                for v in space[n]:
                    cand = dict(best, **{n: v})
                    ts.append((ev(cand), v))
                best[n] = min(ts)[1]
    return [(t, dict(zip(names, k))) for k, t in seen.items()]


def _time(fn, reps):
    best = float("inf")
    for _ in range(reps):
        prep = fn(prepare=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn(prepare=False, state=prep)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return best


def tune_dense(op: str, n: int, reps: int = 2, log=print, spaces=None) -> dict:
    import workloads
    h = cdf.handle()
    # inputs drawn on the GPU (same distributions as the host generators)
    a0 = workloads.lu_uniform_torch(n) if op in ("getrf", "mixed_getrf") else workloads.spd_bbt_torch(n)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    W = cdf.cm_empty(n, n, torch.float32) if op == "mixed_getrf" else None

    def evaluate(params):
        for k, v in params.items():
            h.set_param(k, v)

        def run(prepare, state=None):
            if prepare:
                return a0.clone()
            if op == "getrf":
                cdf.dgetrf(state, ipiv, info)
            elif op == "potrf":
                cdf.dpotrf(state, info)
            else:
                cdf.sgetrf_mixed("bf16", state, W, ipiv, info)

        try:
            t = _time(run, reps)
        finally:
            for k in params:
                h.set_param(k, 0)
        if int(info.item()) != 0:
            t = float("inf")  # a failing candidate is never chosen
        log(f"  {op} n={n} {params}: {t * 1e3:.2f} ms")
        return t

    results = _search(op, evaluate, spaces)
    t, params = min(results, key=lambda r: r[0])
    return {"params": params, "seconds": t, "n": n, "tried": len(results)}


def tune_vbatch(count: int = 4096, dtype: str = "f64", reps: int = 3, log=print, spaces=None) -> dict:
    import workloads
    sizes = workloads.batch_sizes(count)
    kinds = workloads.batch_kinds(count)
    dt = cdf.F64 if dtype == "f64" else cdf.F32
    tdt = torch.float64 if dt == cdf.F64 else torch.float32
    mats = [workloads.batch_problem(i, int(n), int(k)) for i, (n, k) in enumerate(zip(sizes, kinds))]
    offs = np.concatenate([[0], np.cumsum([m.size for m in mats])])
    host = np.concatenate([m.ravel(order="F") for m in mats])
    src = torch.from_numpy(host).to(device="cuda", dtype=tdt)
    buf = torch.empty_like(src)
    es = buf.element_size()
    a_ptrs = torch.tensor([buf.data_ptr() + int(o) * es for o in offs[:-1]], dtype=torch.int64, device="cuda")
    ldas = torch.tensor(sizes, dtype=torch.int32, device="cuda")
    nmax = int(sizes.max())
    piv = torch.zeros((count, nmax), dtype=torch.int32, device="cuda")
    p_ptrs = torch.tensor([piv.data_ptr() + i * nmax * 4 for i in range(count)], dtype=torch.int64, device="cuda")
    info = torch.zeros(count, dtype=torch.int32, device="cuda")
    h = cdf.handle()

    def evaluate(params):
        for k, v in params.items():
            h.set_param(k, v)
        try:
            plan = cdf.VBatchPlan(sizes, kinds, dt, h, tuned=False)
        finally:
            for k in params:
                h.set_param(k, 0)

        def run(prepare, state=None):
            if prepare:
                buf.copy_(src)
                return None
            plan.run(a_ptrs, ldas, p_ptrs, info)

        t = _time(run, reps)
        plan.close()
        log(f"  vbatch {dtype} count={count} {params}: {t * 1e3:.3f} ms")
        return t

    results = _search("vbatch", evaluate, spaces)
    t, params = min(results, key=lambda r: r[0])
    return {"params": params, "seconds": t, "n": int(nmax), "count": count, "tried": len(results)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--op", nargs="+", default=["getrf", "potrf"], choices=list(SPACES))
    ap.add_argument("--n", nargs="+", type=int, default=[8192])
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--dtype", nargs="+", default=["f64"], choices=["f64", "f32"])
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args()
    cache = load_cache(args.cache)
    t0 = time.time()
    for op in args.op:
        if op == "vbatch":
            for dt in args.dtype:
                r = tune_vbatch(args.count, dt, args.reps)
                cache[key(op, dt, r["n"])] = r
                print(f"{op}/{dt}: best {r['params']} {r['seconds'] * 1e3:.3f} ms", flush=True)
        else:
            for n in args.n:
                r = tune_dense(op, n, args.reps)
                cache[key(op, "f64", n)] = r
                print(f"{op}/f64/{n}: best {r['params']} {r['seconds'] * 1e3:.2f} ms", flush=True)
        save_cache(cache, args.cache)
    print(f"tuned in {time.time() - t0:.1f} s -> {args.cache or cache_path()}", flush=True)


if __name__ == "__main__":
    main()
