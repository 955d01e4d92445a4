"""FP64 parity of the HIP path against the CPU oracle (needs an MI355X).

Every call goes through the C-ABI (libcdnafact.so) via the thin binding.
Pivots must be identical to the oracle's; factors agree elementwise within
the rounding-order tolerance of tests/gpu_util.py; the scaled backward error
||PA - LU||_F / (||A||_F n eps) must be <= 10.
"""
import numpy as np
import pytest

import workloads
from tests import golden_cases, gpu_util

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_09337_amd as cdf  # noqa: E402

CASES = golden_cases.load()


def _lu_gpu(a, **params):
    h = cdf.handle()
    for k, v in params.items():
        h.set_param(k, v)
    try:
        A = cdf.to_device(a)
        n = a.shape[0]
        ipiv = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
        info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        cdf.dgetrf(A, ipiv, info)
        torch.cuda.synchronize()
        return cdf.to_host(A), ipiv.cpu().numpy()[:n], int(info.item())
    finally:
        for k in params:
            h.set_param(k, 0)


def _chol_gpu(a, **params):
    h = cdf.handle()
    for k, v in params.items():
        h.set_param(k, v)
    try:
        A = cdf.to_device(a)
        info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        cdf.dpotrf(A, info)
        torch.cuda.synchronize()
        return cdf.to_host(A), int(info.item())
    finally:
        for k in params:
            h.set_param(k, 0)


@pytest.mark.parametrize("name", [n for n, c in CASES.items() if c["kind"] == "lu"])
def test_lu_hand_worked_bitwise(oracle_mod, name):
    c = CASES[name]
    a = golden_cases.as_f64(c["A"])
    lu, ipiv, info = _lu_gpu(a)
    assert list(ipiv) == c["ipiv"] and info == c["info"]
    L, U = oracle_mod.split_lu(lu)
    assert np.array_equal(L, golden_cases.as_f64(c["L"]))
    assert np.array_equal(U, golden_cases.as_f64(c["U"]))


@pytest.mark.parametrize("name", [n for n, c in CASES.items() if c["kind"] == "chol"])
def test_chol_hand_worked_bitwise(oracle_mod, name):
    c = CASES[name]
    a = golden_cases.as_f64(c["A"])
    l, info = _chol_gpu(a)
    assert info == c["info"]
    if not info:
        assert np.array_equal(np.tril(l), golden_cases.as_f64(c["L"]))
    assert np.array_equal(np.triu(l, 1), np.triu(a, 1))


@pytest.mark.parametrize("n,nb", [(1, 0), (2, 0), (3, 0), (31, 0), (32, 0), (33, 0), (100, 0), (255, 0),
                                  (256, 0), (257, 0), (513, 0), (1024, 0), (1500, 0), (700, 64), (700, 96),
                                  (1100, 384), (2100, 512)])
def test_lu_parity_random(oracle_mod, n, nb):
    a = workloads.lu_uniform(n, seed=1000 + n)
    lu_or, ip_or, info_or = oracle_mod.dgetrf(a)
    lu, ip, info = _lu_gpu(a, lu_nb=nb)
    assert info == info_or == 0
    if not np.array_equal(ip, ip_or):
        pytest.fail(gpu_util.first_pivot_mismatch(ip, ip_or, a, oracle_mod))
    tol = gpu_util.lu_parity_tolerance(lu_or)
    assert np.all(np.abs(lu - lu_or) <= tol), float(np.max(np.abs(lu - lu_or) / tol))
    assert np.all(np.abs(np.tril(lu, -1)) <= 1.0)
    assert oracle_mod.lu_backward_error(a, lu, ip) <= 10.0


@pytest.mark.parametrize("rows", [1, 2])
def test_lu_leaf_multi_workgroup(oracle_mod, rows):
    """Tall enough that the panel leaf spreads over many workgroups (grid exchange)."""
    n = 2304
    a = workloads.lu_uniform(n, seed=77)
    lu_or, ip_or, _ = oracle_mod.dgetrf(a)
    lu, ip, info = _lu_gpu(a, lu_leaf_rows=rows)
    assert info == 0
    if not np.array_equal(ip, ip_or):
        pytest.fail(gpu_util.first_pivot_mismatch(ip, ip_or, a, oracle_mod))
    assert oracle_mod.lu_backward_error(a, lu, ip) <= 10.0


def test_lu_parity_n8192_full(oracle_mod):
    """The smallest LU size of the benchmark's size set (n = 8192), whole
    matrix against the oracle: identical pivots, every entry within the
    rounding-order tolerance, backward error <= 10.  The leaf runs with 32
    workgroups at the default parameters."""
    n = 8192
    a = workloads.lu_uniform(n, seed=8192)
    lu_or, ip_or, info_or = oracle_mod.dgetrf(a)
    lu, ip, info = _lu_gpu(a)
    assert info == info_or == 0
    if not np.array_equal(ip, ip_or):
        pytest.fail(gpu_util.first_pivot_mismatch(ip, ip_or, a, oracle_mod))
    # tolerance 16 n eps (|L||U|)_ij (/ |u_jj| for L) with |L||U| from the
    # oracle's factors, formed with torch's FP64 product on the GPU
    Lo = torch.from_numpy(np.tril(lu_or, -1) + np.eye(n)).cuda().abs()
    Uo = torch.from_numpy(np.triu(lu_or)).cuda().abs()
    LU = (Lo @ Uo).cpu().numpy()
    del Lo, Uo
    tol = 16 * n * gpu_util.EPS * LU + 1e-300
    d = np.abs(np.diag(lu_or)).copy()
    low = np.tril(np.ones((n, n), dtype=bool), -1)
    tol[low] = (tol / d[None, :])[low]
    err = np.abs(lu - lu_or)
    assert np.all(err <= tol), float(np.max(err / tol))
    A0 = torch.from_numpy(a).cuda()
    be = gpu_util.lu_backward_error_torch(torch, A0, torch.from_numpy(lu).cuda(), ip)
    assert be <= 10.0, be


def test_chol_parity_n8192_full(oracle_mod):
    """Cholesky at n = 8192, whole lower triangle against the oracle."""
    n = 8192
    a = workloads.spd_bbt(n, seed=8193)
    l_or, info_or = oracle_mod.dpotrf(a)
    l, info = _chol_gpu(a)
    assert info == info_or == 0
    Lo = torch.from_numpy(np.tril(l_or)).cuda().abs()
    LL = (Lo @ Lo.t().contiguous()).cpu().numpy()
    del Lo
    d = np.abs(np.diag(l_or))
    tol = np.tril(16 * n * gpu_util.EPS * LL / d[None, :]) + 1e-300
    err = np.abs(np.tril(l) - np.tril(l_or))
    assert np.all(err <= tol), float(np.max(err / tol))
    assert np.array_equal(np.triu(l, 1), np.triu(a, 1)), "upper triangle was written"
    be = gpu_util.chol_backward_error_torch(torch, torch.from_numpy(a).cuda(), torch.from_numpy(l).cuda())
    assert be <= 10.0, be


@pytest.mark.parametrize("n,k", [(32768, 1024)])
def test_lu_parity_large_first_steps(oracle_mod, n, k):
    """A size of the benchmark's size set (n = 32768) at default parameters:
    512-wide panels, and a leaf grid of 128 workgroups, so every lane of the
    polling wave reads two workgroups' tags.  The oracle factors the first k
    columns plus 256 sampled ones for k steps (the first k steps of
    elimination read nothing else), which fixes the first k pivots, the
    first k columns of L (up to the later interchanges, taken from the GPU's
    pivots) and rows [0, k) of U in the sampled columns.  The whole factor is
    held to the backward-error bound with torch's FP64 products."""
    A0 = workloads.lu_uniform_torch(n, seed=32768)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(np.arange(k, n), 256, replace=False))
    cols = np.concatenate([np.arange(k), sample])
    a_sub = np.asfortranarray(A0[:, torch.from_numpy(cols).cuda()].cpu().numpy())
    A = cdf.cm_empty(n, n)
    A.copy_(A0)
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    cdf.dgetrf(A, ipiv, info)
    assert cdf.device_status() == cdf.CDF_OK
    assert int(info.item()) == 0
    ip = ipiv.cpu().numpy()
    lu_k, ip_k, info_k = oracle_mod.dgetrf(a_sub, ksteps=k)
    assert info_k == 0
    if not np.array_equal(ip[:k], ip_k[:k]):
        j = int(np.nonzero(ip[:k] != ip_k[:k])[0][0])
        part, _, _ = oracle_mod.dgetrf(np.asfortranarray(a_sub[:, :j + 1]), ksteps=j)
        col = np.abs(part[j:, j])
        g, o = int(ip[j]) - 1 - j, int(ip_k[j]) - 1 - j
        pytest.fail(f"step {j}: gpu row {g + j} |a|={col[g]!r}, oracle row {o + j} |a|={col[o]!r}")
    tol = gpu_util.lu_partial_tolerance(lu_k, k, n)
    # the GPU's later interchanges (steps >= k) also moved rows of L[:, :k]
    perm = gpu_util.perm_from_ipiv(np.concatenate([np.arange(1, k + 1), ip[k:]]), n)
    got = np.zeros((n, k + len(sample)))
    got[:, :k] = A[:, :k].cpu().numpy()
    got[:k, k:] = A[:k, torch.from_numpy(sample).cuda()].cpu().numpy()
    want = lu_k.copy()
    want[:, :k] = want[perm, :k]
    tol[:, :k] = tol[perm, :k]
    err = np.abs(got - want)
    assert np.all(err <= tol), float(np.nanmax(np.where(np.isfinite(tol), err / tol, 0.0)))
    be = gpu_util.lu_backward_error_torch(torch, A0, A, ip)
    assert be <= 10.0, be


@pytest.mark.parametrize("n,nb", [(1300, 256), (600, 64)])
def test_lu_exchange_timeout_returns(oracle_mod, n, nb):
    """The leaf's grid-exchange waits are bounded.  With the testing switch
    that makes every wait of a multi-workgroup leaf wait for a tag nobody
    writes, each wait gives up after its budget (200 us here): info reads
    CDF_INFO_TIMEOUT, cdf_device_status reports CDF_ERR_TIMEOUT, the pivots
    stay in range, and every kernel of the call ends.  The same handle then
    factors normally, matching the oracle."""
    a = workloads.lu_uniform(n, seed=91)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = cdf.handle()
        h.set_param("lu_nb", nb)
        h.set_param("leaf_wait_us", 200)
        h.set_param("test_exchange_fail", 1)
        A = cdf.to_device(a)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        cdf.dgetrf(A, ipiv, info, h)
        assert cdf.device_status(h) == cdf.CDF_ERR_TIMEOUT
        assert int(info.item()) == cdf.CDF_INFO_TIMEOUT
        ip = ipiv.cpu().numpy()
        assert np.all((ip >= np.arange(1, n + 1)) & (ip <= n))
        h.set_param("test_exchange_fail", 0)
        h.set_param("leaf_wait_us", 0)
        A = cdf.to_device(a)
        info.fill_(-7)
        cdf.dgetrf(A, ipiv, info, h)
        assert cdf.device_status(h) == cdf.CDF_OK
        lu, ip = cdf.to_host(A), ipiv.cpu().numpy()
        h.set_param("lu_nb", 0)
    assert int(info.item()) == 0
    lu_or, ip_or, _ = oracle_mod.dgetrf(a)
    assert np.array_equal(ip, ip_or)
    tol = gpu_util.lu_parity_tolerance(lu_or)
    assert np.all(np.abs(lu - lu_or) <= tol)


def test_lu_exchange_timeout_mixed_lu():
    """The mixed-precision LU runs the same leaf: a forced exchange timeout
    comes back from the solver as CDF_ERR_TIMEOUT."""
    n = 700
    a = workloads.diag_dominant(n, seed=3)
    b = workloads.rhs_uniform(n, 1, seed=4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = cdf.handle()
        h.set_param("leaf_wait_us", 200)
        h.set_param("test_exchange_fail", 1)
        A, B = cdf.to_device(a), cdf.to_device(b)
        X = torch.empty_like(B)
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        with pytest.raises(cdf.CdfError) as e:
            cdf.dgesv_mixed("bf16", A, B, X, info, h=h)
        assert e.value.status == cdf.CDF_ERR_TIMEOUT
        h.set_param("test_exchange_fail", 0)
        h.set_param("leaf_wait_us", 0)
        r = cdf.dgesv_mixed("bf16", A, B, X, info, h=h)
    assert r["converged"] and r["scaled_resid"] <= 16


@pytest.mark.parametrize("nb", [64, 256])
def test_lu_exact_factors(oracle_mod, nb):
    """A = L U with small dyadic L and integer U (identity pivots): formed by
    substitution, U12 and hence both factors come back exactly.  This L is
    very ill-conditioned across blocks (|L^-1| ~ 1e12 over 512 rows), so one
    rounding error in U12 (an accepted L11^-1) grows through the later blocks:
    the default path is held to the backward error, and where the guard
    rejects every L11^-1 (nb = 256) to exactness."""
    n = 700
    rng = np.random.default_rng(nb)
    L = np.tril(rng.integers(-2, 3, (n, n)) / 4.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-4, 5, (n, n)).astype(np.float64))
    U[np.diag_indices(n)] = rng.choice([-1.0, 1.0], n) * rng.integers(16, 32, n)
    a = np.asfortranarray(L @ U)
    lu, ip, info = _lu_gpu(a, lu_nb=nb, lu_u12=1)
    assert info == 0 and np.array_equal(ip, np.arange(1, n + 1))
    assert np.array_equal(np.tril(lu, -1) + np.eye(n), L) and np.array_equal(np.triu(lu), U)
    lu2, ip2, info2 = _lu_gpu(a, lu_nb=nb)
    assert info2 == 0 and np.array_equal(ip2, ip)
    assert oracle_mod.lu_backward_error(a, lu2, ip2) <= 10.0
    if nb == 256:
        # |L11^-1| reaches ~1e6 for these 256-wide blocks: the guard rejects
        # every inverse and the default path solves by substitution, exactly
        assert np.array_equal(lu2, lu)


def test_lu_guard_fallback_wide_exact():
    """Every L11^-1 of this L is rejected by the guard; the fallback
    substitution runs on a capped grid whose workgroups loop over more than
    one column block each (over 8192 trailing columns): factors exact."""
    n, nb = 8960, 256
    rng = np.random.default_rng(3)
    L = np.tril(rng.integers(-2, 3, (n, n)) / 4.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-4, 5, (n, n)).astype(np.float64))
    U[np.diag_indices(n)] = rng.choice([-1.0, 1.0], n) * rng.integers(16, 32, n)
    a = np.asfortranarray(L @ U)
    lu, ip, info = _lu_gpu(a, lu_nb=nb)
    assert info == 0 and np.array_equal(ip, np.arange(1, n + 1))
    assert np.array_equal(np.tril(lu, -1) + np.eye(n), L) and np.array_equal(np.triu(lu), U)


def test_lu_in_place_u12_under_workspace_cap(oracle_mod):
    """Capped below U12's buffer, the LU solves U12 in place (blocked substitution)
    instead of through L11^-1: same pivots as the oracle, same tolerance."""
    n = 1300
    a = workloads.lu_uniform(n, seed=4242)
    lu_or, ip_or, _ = oracle_mod.dgetrf(a)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = cdf.handle()  # a fresh handle: its workspace starts empty
        h.set_workspace_limit(4 << 20)
        h.set_param("lu_nb", 256)
        A = cdf.to_device(a)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        cdf.dgetrf(A, ipiv, info, h)
        torch.cuda.synchronize()
        assert h.workspace_bytes() <= 4 << 20
        lu, ip = cdf.to_host(A), ipiv.cpu().numpy()
    assert int(info.item()) == 0
    if not np.array_equal(ip, ip_or):
        pytest.fail(gpu_util.first_pivot_mismatch(ip, ip_or, a, oracle_mod))
    tol = gpu_util.lu_parity_tolerance(lu_or)
    assert np.all(np.abs(lu - lu_or) <= tol), float(np.max(np.abs(lu - lu_or) / tol))
    assert oracle_mod.lu_backward_error(a, lu, ip) <= 10.0


def test_lu_singular_info(oracle_mod):
    n = 300
    a = workloads.lu_uniform(n, seed=5)
    a[:, 137] = 0.0  # exactly zero column -> first zero pivot at step 137
    _, ip_or, info_or = oracle_mod.dgetrf(a)
    lu, ip, info = _lu_gpu(a)
    assert info == info_or == 138
    assert np.array_equal(ip, ip_or)
    z = np.zeros((40, 40), order="F")
    _, ipz, infoz = _lu_gpu(z)
    assert infoz == 1 and np.array_equal(ipz, np.arange(1, 41))


def test_lu_diag_dominant_identity_pivots():
    a = workloads.diag_dominant(600, seed=0)
    _, ip, info = _lu_gpu(a)
    assert info == 0 and np.array_equal(ip, np.arange(1, 601))


@pytest.mark.parametrize("n,nrhs", [(1, 1), (300, 1), (1024, 1), (4100, 4), (2000, 2), (777, 5), (1024, 64)])
def test_getrs(oracle_mod, n, nrhs):
    a = workloads.lu_uniform(n, seed=n)
    b = workloads.rhs_uniform(n, nrhs, seed=n + 1)
    lu_or, ip_or, _ = oracle_mod.dgetrf(a)
    x_or = oracle_mod.dgetrs(lu_or, ip_or, b)
    A = cdf.to_device(a)
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    cdf.dgetrf(A, ipiv, info)
    B = cdf.to_device(b)
    cdf.dgetrs(A, ipiv, B)
    x = cdf.to_host(B)
    assert oracle_mod.hpl_scaled_residual(a, x, b) <= 16
    kappa = np.linalg.cond(a, np.inf)
    assert np.max(np.abs(x - x_or)) <= 2 * 16 * n * oracle_mod.EPS * kappa * np.max(np.abs(x_or))


@pytest.mark.parametrize("n,nb", [(1, 0), (2, 0), (5, 0), (64, 0), (127, 0), (128, 0), (129, 0), (400, 0),
                                  (1000, 0), (1300, 64), (700, 96), (1500, 256), (900, 384), (1300, 512)])
def test_chol_parity_random(oracle_mod, n, nb):
    a = workloads.spd_bbt(n, seed=2000 + n)
    l_or, info_or = oracle_mod.dpotrf(a)
    l, info = _chol_gpu(a, chol_nb=nb)
    assert info == info_or == 0
    tol = gpu_util.chol_parity_tolerance(l_or)
    d = np.abs(np.tril(l) - np.tril(l_or))
    assert np.all(d <= tol), float(np.max(d / tol))
    assert np.array_equal(np.triu(l, 1), np.triu(a, 1)), "upper triangle was written"
    assert oracle_mod.chol_backward_error(a, l) <= 10.0


@pytest.mark.parametrize("n,bad,nb", [(300, 0, 0), (300, 150, 0), (300, 299, 0), (260, 128, 0), (600, 200, 256),
                                      (700, 450, 512)])
def test_chol_not_spd_info(oracle_mod, n, bad, nb):
    a = workloads.spd_bbt(n, seed=3)
    a[bad, bad] = -1.0
    _, info_or = oracle_mod.dpotrf(a)
    l, info = _chol_gpu(a, chol_nb=nb)
    assert info == info_or
    # columns of finished blocks before the failing one agree with the oracle
    lo, _ = oracle_mod.dpotrf(a, ksteps=(bad // 128) * 128)
    k = (bad // 128) * 128
    assert np.allclose(np.tril(l)[:, :k], np.tril(lo)[:, :k], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,nrhs", [(1, 1), (500, 1), (1024, 64), (333, 3), (3001, 4)])
def test_potrs(oracle_mod, n, nrhs):
    a = workloads.spd_bbt(n, seed=n)
    b = workloads.rhs_uniform(n, nrhs, seed=n + 2)
    l_or, _ = oracle_mod.dpotrf(a)
    x_or = oracle_mod.dpotrs(l_or, b)
    A = cdf.to_device(a)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    cdf.dpotrf(A, info)
    B = cdf.to_device(b)
    cdf.dpotrs(A, B)
    x = cdf.to_host(B)
    assert oracle_mod.hpl_scaled_residual(a, x, b) <= 16
    assert np.max(np.abs(x - x_or)) <= 1e-12 * np.max(np.abs(x_or)) * n


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (128, 128, 16), (129, 130, 17), (300, 77, 256), (1000, 1000, 256),
                                   (17, 513, 5)])
def test_dgemm_update(m, n, k):
    rng = np.random.default_rng(m * 7 + n + k)
    a = np.asfortranarray(rng.uniform(-1, 1, (m, k)))
    b = np.asfortranarray(rng.uniform(-1, 1, (k, n)))
    c = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    C = cdf.to_device(c)
    cdf.dgemm_update(cdf.to_device(a), cdf.to_device(b), C)
    ref = c - a @ b
    got = cdf.to_host(C)
    assert np.max(np.abs(got - ref)) <= 4 * k * gpu_util.EPS * (np.abs(a) @ np.abs(b) + np.abs(c)).max()


@pytest.mark.parametrize("m,n,k", [(1000, 700, 512), (130, 66, 48), (64, 1, 16)])
def test_dgemm_update_fast_path_matches_general_path(m, n, k):
    """Aligned even shapes take the direct-to-LDS kernel; the same product with
    an odd leading dimension for A takes the general kernel.  Both accumulate
    in the same order, so the results must agree bit for bit."""
    rng = np.random.default_rng(m + 3 * n + k)
    a = rng.uniform(-1, 1, (m, k))
    b = np.asfortranarray(rng.uniform(-1, 1, (k, n)))
    c = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    A_even = cdf.to_device(np.asfortranarray(a))
    A_odd_store = cdf.cm_empty(m + 1, k)             # leading dimension m + 1 (odd)
    A_odd_store[:m].copy_(A_even)
    A_odd = A_odd_store[:m]
    B = cdf.to_device(b)
    C1, C2 = cdf.to_device(c), cdf.to_device(c)
    cdf.dgemm_update(A_even, B, C1)
    cdf.dgemm_update(A_odd, B, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    ref = c - a @ b
    assert np.max(np.abs(cdf.to_host(C1) - ref)) <= 4 * k * gpu_util.EPS * (np.abs(a) @ np.abs(b) + np.abs(c)).max()


@pytest.mark.parametrize("m,n,k", [(1000, 700, 512), (130, 258, 48), (2050, 130, 16), (384, 384, 64)])
def test_dgemm_tile128_matches_tile64(m, n, k):
    """The 128 x 128-tile update GEMM accumulates every entry in the same
    order as the 64 x 64 one (K steps of 16, MFMA k-groups of 4): results
    agree bit for bit, on ragged shapes too."""
    rng = np.random.default_rng(m + 7 * n + k)
    a = np.asfortranarray(rng.uniform(-1, 1, (m, k)))
    b = np.asfortranarray(rng.uniform(-1, 1, (k, n)))
    c = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    h = cdf.handle()
    out = {}
    try:
        for tile in (64, 128):
            h.set_param("gemm_tile", tile)
            C = cdf.to_device(c)
            cdf.dgemm_update(cdf.to_device(a), cdf.to_device(b), C)
            torch.cuda.synchronize()
            out[tile] = C
    finally:
        h.set_param("gemm_tile", 0)
    assert torch.equal(out[64], out[128])
    ref = c - a @ b
    assert np.max(np.abs(cdf.to_host(out[128]) - ref)) <= 4 * k * gpu_util.EPS * (np.abs(a) @ np.abs(b) + np.abs(c)).max()


@pytest.mark.parametrize("n,nb", [(2100, 512), (1500, 256)])
def test_lu_parity_tile128(oracle_mod, n, nb):
    """LU with every large-enough update on 128 x 128 tiles."""
    a = workloads.lu_uniform(n, seed=4000 + n)
    lu_or, ip_or, info_or = oracle_mod.dgetrf(a)
    lu, ip, info = _lu_gpu(a, lu_nb=nb, gemm_tile=128)
    assert info == info_or == 0
    if not np.array_equal(ip, ip_or):
        pytest.fail(gpu_util.first_pivot_mismatch(ip, ip_or, a, oracle_mod))
    tol = gpu_util.lu_parity_tolerance(lu_or)
    assert np.all(np.abs(lu - lu_or) <= tol), float(np.max(np.abs(lu - lu_or) / tol))
    assert oracle_mod.lu_backward_error(a, lu, ip) <= 10.0


def test_invalid_arguments():
    h = cdf.handle()
    L = cdf.lib()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = L.cdf_dgetrf(h.bind_stream(), -1, None, 1, None, cdf._p(info))
    assert st == cdf.CDF_ERR_INVALID_ARG and L.cdf_last_bad_arg(h.ptr) == 2
    A = cdf.cm_empty(4, 4)
    st = L.cdf_dgetrf(h.bind_stream(), 4, cdf._p(A), 3, cdf._p(info), cdf._p(info))
    assert st == cdf.CDF_ERR_INVALID_ARG and L.cdf_last_bad_arg(h.ptr) == 4
    st = L.cdf_dpotrf(h.bind_stream(), b"U", 4, cdf._p(A), 4, cdf._p(info))
    assert st == cdf.CDF_ERR_UNSUPPORTED
    st = L.cdf_dpotrf(h.bind_stream(), b"X", 4, cdf._p(A), 4, cdf._p(info))
    assert st == cdf.CDF_ERR_INVALID_ARG and L.cdf_last_bad_arg(h.ptr) == 2
    st = L.cdf_dgetrs(h.bind_stream(), b"N", 4, -2, cdf._p(A), 4, cdf._p(info), cdf._p(A), 4)
    assert st == cdf.CDF_ERR_INVALID_ARG and L.cdf_last_bad_arg(h.ptr) == 4
    # n = 0 is a no-op that reports info = 0
    info.fill_(5)
    assert L.cdf_dgetrf(h.bind_stream(), 0, None, 1, None, cdf._p(info)) == cdf.CDF_OK
    torch.cuda.synchronize()
    assert info.item() == 0
    with pytest.raises(cdf.CdfError):
        h.set_param("lu_nb", 33)
    for name, bad_values in (("gemm_wg_per_cu", (1, 2, 6)), ("lu_u12", (2, -1))):
        for v in bad_values:
            with pytest.raises(cdf.CdfError):
                h.set_param(name, v)
        assert h.get_param(name) == 0
    for v in (3, 4, 5, 0):
        h.set_param("gemm_wg_per_cu", v)
        assert h.get_param("gemm_wg_per_cu") == v
