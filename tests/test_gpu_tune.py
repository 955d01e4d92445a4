"""The autotuner on the GPU: it searches small getrf / potrf / mixed-LU
spaces at n = 2048 and a 300-problem batch, writes a cache that reads back
unchanged, the chosen parameters are what apply() sets on a handle (and
what the batched plan takes by itself), and factorizations with them stay
parity-green against the oracle."""
import json

import numpy as np
import pytest
import torch

import paper_2108_09337_amd as cdf
import workloads
from paper_2108_09337_amd import tune
from tests import gpu_util
from tests.test_gpu_vbatch import make_batch, unpack

pytestmark = pytest.mark.gpu

SMALL = {  # reduced spaces: every dimension still searched
    "getrf": {"lu_nb": [128, 256], "lu_leaf_rows": [1, 2], "gemm_wg_per_cu": [4, 5], "gemm_tile": [64, 128],
              "lu_u12": [0, 1]},
    "potrf": {"chol_nb": [128, 256], "gemm_wg_per_cu": [4, 5]},
    "mixed_getrf": {"mixed_nb": [256], "lu_u12": [0, 1], "lu_pivot": [0, 1]},
    "vbatch": {"vbatch_nb": [0, 16], "vbatch_wg_per_cu": [1, 2]},
}


@pytest.fixture
def cache_file(tmp_path):
    return str(tmp_path / "tune_cache.json")


def _roundtrip(cache_file, cache):
    tune.save_cache(cache, cache_file)
    back = tune.load_cache(cache_file)
    assert back == json.loads(json.dumps(cache))
    return back


def test_tune_dense_and_apply(oracle_mod, cache_file):
    n = 2048
    cache = {}
    for op in ("getrf", "potrf", "mixed_getrf"):
        print(f"tuning {op} n={n}", flush=True)
        r = tune.tune_dense(op, n, reps=1, log=lambda *a: None, spaces=SMALL)
        for k, v in r["params"].items():
            assert v in SMALL[op][k]
        assert r["tried"] >= 2 and np.isfinite(r["seconds"])
        cache[tune.key(op, "f64", n)] = r
    back = _roundtrip(cache_file, cache)
    h = cdf.handle()
    a = workloads.lu_uniform(n, seed=3)
    s = workloads.spd_bbt(n, seed=4)
    try:
        p = tune.apply(h, "getrf", n, cache=back)
        for k, v in p.items():
            assert h.get_param(k) == v
        A = cdf.to_device(a)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.full((1,), -3, dtype=torch.int32, device="cuda")
        cdf.dgetrf(A, ipiv, info)
        torch.cuda.synchronize()
        lu, ip = cdf.to_host(A), ipiv.cpu().numpy()
        lu_or, ip_or, _ = oracle_mod.dgetrf(a)
        assert int(info.item()) == 0 and np.array_equal(ip, ip_or)
        assert np.all(np.abs(lu - lu_or) <= gpu_util.lu_parity_tolerance(lu_or))
        for k in p:
            h.set_param(k, 0)
        p = tune.apply(h, "potrf", n, cache=back)
        S = cdf.to_device(s)
        cdf.dpotrf(S, info)
        torch.cuda.synchronize()
        l_or, _ = oracle_mod.dpotrf(s)
        L = np.tril(cdf.to_host(S))
        assert int(info.item()) == 0
        assert np.all(np.abs(L - np.tril(l_or)) <= gpu_util.chol_parity_tolerance(l_or))
    finally:
        for k in ("lu_nb", "lu_leaf_rows", "gemm_wg_per_cu", "gemm_tile", "lu_u12", "chol_nb", "lu_pivot",
                  "mixed_nb"):
            h.set_param(k, 0)


def test_tune_vbatch_and_plan(oracle_mod, cache_file, monkeypatch):
    count = 300
    r = tune.tune_vbatch(count, "f64", reps=1, log=lambda *a: None, spaces=SMALL)
    assert r["tried"] == 4
    cache = {tune.key("vbatch", "f64", r["n"]): r}
    _roundtrip(cache_file, cache)
    monkeypatch.setenv("CDF_TUNE_CACHE", cache_file)
    sizes = workloads.batch_sizes(count)
    kinds = workloads.batch_kinds(count)
    h = cdf.handle()
    before = {k: h.get_param(k) for k in SMALL["vbatch"]}
    plan = cdf.VBatchPlan(sizes, kinds, cdf.F64, h)
    assert plan.params == r["params"]
    assert {k: h.get_param(k) for k in SMALL["vbatch"]} == before  # the handle is left as it was
    mats, buf, offs, a_ptrs, ldas, piv, p_ptrs, info = make_batch(sizes, kinds, cdf.F64)
    plan.run(a_ptrs, ldas, p_ptrs, info)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    piv_h = piv.cpu().numpy()
    for i in range(count):
        n = int(sizes[i])
        f = unpack(buf, offs, sizes, i)
        if kinds[i] == 0:
            lu_or, ip_or, _ = oracle_mod.dgetrf(mats[i])
            assert np.array_equal(piv_h[i, :n], ip_or), i
            assert np.all(np.abs(f - lu_or) <= gpu_util.lu_parity_tolerance(lu_or)), i
        else:
            l_or, _ = oracle_mod.dpotrf(mats[i])
            assert np.all(np.abs(np.tril(f) - np.tril(l_or)) <= gpu_util.chol_parity_tolerance(l_or)), i
    plan.close()
