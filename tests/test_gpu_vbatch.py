"""Batched small factorizations (one persistent launch) against the
per-problem CPU oracle (needs an MI355X)."""
import numpy as np
import pytest

import workloads
from tests import gpu_util

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_09337_amd as cdf  # noqa: E402


def make_batch(sizes, kinds, dtype, seed=0):
    """Matrices of the batched workload packed in one device buffer."""
    mats = [workloads.batch_problem(i, int(n), int(k), seed=seed) for i, (n, k) in enumerate(zip(sizes, kinds))]
    tdt = torch.float64 if dtype == cdf.F64 else torch.float32
    offs = np.concatenate([[0], np.cumsum([m.size for m in mats])])
    buf = torch.empty(int(offs[-1]), dtype=tdt, device="cuda")
    for m, o in zip(mats, offs[:-1]):
        buf[int(o):int(o) + m.size].copy_(torch.from_numpy(m.ravel(order="F")).to(tdt))
    es = buf.element_size()
    base = buf.data_ptr()
    a_ptrs = torch.tensor([base + int(o) * es for o in offs[:-1]], dtype=torch.int64, device="cuda")
    ldas = torch.tensor([int(n) for n in sizes], dtype=torch.int32, device="cuda")
    nmax = int(max(sizes))
    piv = torch.zeros((len(sizes), nmax), dtype=torch.int32, device="cuda")
    p_ptrs = torch.tensor([piv.data_ptr() + i * nmax * 4 for i in range(len(sizes))], dtype=torch.int64, device="cuda")
    info = torch.full((len(sizes),), -5, dtype=torch.int32, device="cuda")
    return mats, buf, offs, a_ptrs, ldas, piv, p_ptrs, info


def unpack(buf, offs, sizes, i):
    n = int(sizes[i])
    a = buf[int(offs[i]):int(offs[i]) + n * n].double().cpu().numpy()
    return a.reshape(n, n, order="F")


@pytest.mark.parametrize("count,dt", [(300, cdf.F64), (300, cdf.F32), (4096, cdf.F64)])
def test_vbatch_against_oracle(oracle_mod, count, dt):
    sizes = workloads.batch_sizes(count)
    kinds = workloads.batch_kinds(count)
    mats, buf, offs, a_ptrs, ldas, piv, p_ptrs, info = make_batch(sizes, kinds, dt)
    plan = cdf.VBatchPlan(sizes, kinds, dt)
    plan.run(a_ptrs, ldas, p_ptrs, info)
    torch.cuda.synchronize()
    info_h = info.cpu().numpy()
    piv_h = piv.cpu().numpy()
    assert np.all(info_h == 0)
    eps = 2.0 ** -53 if dt == cdf.F64 else 2.0 ** -24
    check = range(count) if count <= 300 else np.random.default_rng(0).choice(count, 200, replace=False)
    for i in check:
        n = int(sizes[i])
        a = mats[i]
        f = unpack(buf, offs, sizes, i)
        if kinds[i] == 0:
            ip = piv_h[i, :n]
            L, U = oracle_mod.split_lu(f)
            p = oracle_mod.ipiv_to_perm(ip, n)
            a_used = a.astype(np.float32).astype(np.float64) if dt == cdf.F32 else a
            be = np.linalg.norm(a_used[p] - L @ U) / (np.linalg.norm(a_used) * n * eps)
            assert be <= 10, (i, n, be)
            assert np.all(np.abs(np.tril(f, -1)) <= 1.0)
            if dt == cdf.F64:
                lu_or, ip_or, _ = oracle_mod.dgetrf(a)
                if not np.array_equal(ip, ip_or):
                    pytest.fail(f"problem {i}: " + gpu_util.first_pivot_mismatch(ip, ip_or, a, oracle_mod))
                tol = gpu_util.lu_parity_tolerance(lu_or)
                assert np.all(np.abs(f - lu_or) <= tol), (i, n)
        else:
            a_used = a.astype(np.float32).astype(np.float64) if dt == cdf.F32 else a
            Lc = np.tril(f)
            be = np.linalg.norm(np.tril(a_used) + np.tril(a_used, -1).T - Lc @ Lc.T) / (
                np.linalg.norm(a_used) * n * eps)
            assert be <= 10, (i, n, be)
            assert np.array_equal(np.triu(f, 1), np.triu(a_used, 1)), "upper triangle written"
            if dt == cdf.F64:
                l_or, _ = oracle_mod.dpotrf(a)
                tol = gpu_util.chol_parity_tolerance(l_or)
                assert np.all(np.abs(np.tril(f) - np.tril(l_or)) <= tol), (i, n)
    plan.close()


def test_vbatch_replay_is_deterministic_and_rebinds_pointers():
    count = 200
    sizes = workloads.batch_sizes(count, seed=9)
    kinds = workloads.batch_kinds(count)
    plan = cdf.VBatchPlan(sizes, kinds, cdf.F64)
    first = make_batch(sizes, kinds, cdf.F64, seed=1)
    second = make_batch(sizes, kinds, cdf.F64, seed=1)
    other = make_batch(sizes, kinds, cdf.F64, seed=2)
    for b in (first, second, other):
        plan.run(b[3], b[4], b[6], b[7])
        torch.cuda.synchronize()
    assert torch.equal(first[1], second[1]) and torch.equal(first[5], second[5])
    assert not torch.equal(first[1], other[1])
    assert int(other[7].abs().sum().item()) == 0


def test_vbatch_singular_and_not_spd_info(oracle_mod):
    sizes = np.array([40, 70, 33, 100], dtype=np.int32)
    kinds = np.array([0, 1, 0, 1], dtype=np.int32)
    mats, buf, offs, a_ptrs, ldas, piv, p_ptrs, info = make_batch(sizes, kinds, cdf.F64, seed=3)
    m0 = mats[0].copy()
    m0[:, 17] = 0.0
    m1 = mats[1].copy()
    m1[50, 50] = -1.0
    for i, m in ((0, m0), (1, m1)):
        buf[int(offs[i]):int(offs[i]) + m.size].copy_(torch.from_numpy(m.ravel(order="F")))
    plan = cdf.VBatchPlan(sizes, kinds, cdf.F64)
    plan.run(a_ptrs, ldas, p_ptrs, info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    assert inf[0] == oracle_mod.dgetrf(m0)[2] == 18
    assert inf[1] == oracle_mod.dpotrf(m1)[1]
    assert inf[2] == 0 and inf[3] == 0


def test_vbatch_invalid_sizes():
    h = cdf.handle()
    with pytest.raises(cdf.CdfError):
        cdf.VBatchPlan(np.array([10, 2000]), np.array([0, 1]), cdf.F64, h)
    with pytest.raises(cdf.CdfError):
        cdf.VBatchPlan(np.array([10, 20]), np.array([0, 3]), cdf.F64, h)
