"""Mixed-precision path on the GPU against the CPU oracle (needs an MI355X).

* quantizer: bit-exact codes and tile exponents;
* low-precision update: exact on exactly representable operands, within the
  binary32 accumulation bound otherwise;
* mixed factorizations: exact on exactly representable factors, elementwise
  close to the oracle's mixed factorization otherwise;
* refinement: HPL scaled residual <= 16 and forward error against the FP64
  oracle solution.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_09337_amd as cdf  # noqa: E402

FMTS = ["bf16", "fp16", "e4m3"]
U32 = 2.0 ** -24
UFMT = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "e4m3": 2.0 ** -4}


def _codes_dtype(fmt):
    return torch.uint8 if fmt == "e4m3" else torch.int16


def _quantize_gpu(fmt, x, tm, tn, ldq=None):
    m, n = x.shape
    ldq = ldq or m
    X = cdf.to_device(x, dtype=torch.float32)
    Q = torch.zeros((n, ldq), dtype=_codes_dtype(fmt), device="cuda")  # column-major, ld = ldq
    mt, nt = -(-m // tm), -(-n // tn)
    E = torch.full((mt * nt,), -999, dtype=torch.int32, device="cuda")
    h = cdf.handle()
    st = cdf.lib().cdf_quantize(h.bind_stream(), cdf.UPD[fmt], m, n, cdf._p(X), cdf._ld(X), tm, tn, cdf._p(Q), ldq,
                                cdf._p(E))
    assert st == 0, st
    torch.cuda.synchronize()
    q = Q.cpu().numpy()
    if fmt != "e4m3":
        q = q.view(np.uint16)
    return q.T.copy(order="F"), E.cpu().numpy().reshape(nt, mt).T


def _spread(rng, shape, lo=-20, hi=20):
    return (rng.choice([-1.0, 1.0], shape) * np.exp(rng.uniform(lo, hi, shape))).astype(np.float32)


@pytest.mark.parametrize("fmt", FMTS)
def test_quantize_bitexact(oracle_mod, fmt):
    rng = np.random.default_rng(42)
    m, n, tm, tn = 300, 200, 128, 64
    x = rng.standard_normal((m, n)).astype(np.float32)
    x[:128, :64] = _spread(rng, (128, 64))                      # wide dynamic range
    x[128:256, 64:128] = 0.0                                     # all-zero tile
    x[:128, 128:192] *= 1e6                                      # amax above maxfinite (negative scale)
    x[256:, 128:192] = _spread(rng, (44, 64), -40, -20)          # tiny values
    # exact ties at the format's rounding midpoints in the (0, 0) tile of the last columns
    table = oracle_mod.decode_table(oracle_mod.FMT_NAMES[fmt])
    fin = np.sort(table[np.isfinite(table) & (table > 0)])
    mids = 0.5 * (fin[:-1] + fin[1:])
    top = {"bf16": 3e38, "fp16": 65504.0, "e4m3": 448.0}[fmt]
    mids = mids[(mids < top) & (mids > 1e-30)]
    k = min(128 * 8, len(mids))
    blk = np.zeros((128, 8), np.float32)
    sel = rng.choice(len(mids), k, replace=False)
    blk.flat[:k] = mids[sel].astype(np.float32)
    blk[0, 0] = np.float32(top if fmt != "bf16" else 1.0)      # pins the tile exponent to 0
    x[:128, 192:200] = blk
    ldq = 320
    q, e = _quantize_gpu(fmt, x, tm, tn, ldq)
    q_or, e_or = oracle_mod.quantize(oracle_mod.FMT_NAMES[fmt], x, tm, tn)
    assert np.array_equal(e, e_or)
    assert np.array_equal(q[:m], q_or), np.argwhere(q[:m] != q_or)[:5]
    assert not np.any(q[m:]), "padding rows must hold zero codes"


def _lowp_gpu(fmt, a, b, c, h=None):
    """C - dq(A) dq(B) through cdf_quantize (of A^T and B) + cdf_lowp_update."""
    m, k = a.shape
    n = b.shape[1]
    T = cdf.update_tile(fmt)
    kp = -(-k // 32) * 32
    qa, ea = _quantize_gpu(fmt, np.asfortranarray(a.T), k, T, kp)
    qb, eb = _quantize_gpu(fmt, b, k, T, kp)
    dt = _codes_dtype(fmt)
    QA = torch.from_numpy(np.ascontiguousarray(qa.T).view(np.int16) if fmt != "e4m3" else np.ascontiguousarray(qa.T)).to("cuda")
    QB = torch.from_numpy(np.ascontiguousarray(qb.T).view(np.int16) if fmt != "e4m3" else np.ascontiguousarray(qb.T)).to("cuda")
    EA = torch.from_numpy(np.ascontiguousarray(ea.ravel(order="F"))).to("cuda")
    EB = torch.from_numpy(np.ascontiguousarray(eb.ravel(order="F"))).to("cuda")
    assert QA.dtype == dt and QB.dtype == dt
    C = cdf.to_device(c, dtype=torch.float32)
    hh = cdf.handle()
    st = cdf.lib().cdf_lowp_update(hh.bind_stream(), cdf.UPD[fmt], m, n, k, cdf._p(QA), kp, cdf._p(EA), cdf._p(QB),
                                   kp, cdf._p(EB), cdf._p(C), cdf._ld(C))
    assert st == 0, st
    torch.cuda.synchronize()
    return cdf.to_host(C).astype(np.float64), (qa, ea, qb, eb)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("m,n,k", [(128, 128, 32), (300, 257, 100), (64, 600, 256), (522, 384, 1000)])
def test_lowp_update_exact_on_representable(fmt, m, n, k):
    rng = np.random.default_rng(m + n + k)
    a = rng.integers(-8, 9, (m, k)).astype(np.float32)
    b = rng.integers(-8, 9, (k, n)).astype(np.float32)
    c = rng.integers(-1000, 1000, (m, n)).astype(np.float32)
    got, _ = _lowp_gpu(fmt, np.asfortranarray(a), np.asfortranarray(b), np.asfortranarray(c))
    assert np.array_equal(got, c.astype(np.float64) - a.astype(np.float64) @ b.astype(np.float64))


@pytest.mark.parametrize("fmt", FMTS)
def test_lowp_update_random(oracle_mod, fmt):
    rng = np.random.default_rng(3)
    m, n, k = 333, 290, 200
    a = np.asfortranarray(rng.uniform(-1, 1, (m, k)).astype(np.float32))
    b = np.asfortranarray((rng.uniform(-1, 1, (k, n)) * 30).astype(np.float32))
    c = np.asfortranarray(rng.uniform(-50, 50, (m, n)).astype(np.float32))
    got, (qa, ea, qb, eb) = _lowp_gpu(fmt, a, b, c)
    f = oracle_mod.FMT_NAMES[fmt]
    T = cdf.update_tile(fmt)
    da = oracle_mod.dequantize(f, qa[:k], ea, k, T).T          # exact dq(A)
    db = oracle_mod.dequantize(f, qb[:k], eb, k, T)
    ref = c.astype(np.float64) - da @ db
    bound = (k + 2) * U32 * (np.abs(c) + np.abs(da) @ np.abs(db))
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))


def _exact_lu(n, rng):
    L = np.tril(rng.integers(-2, 3, (n, n)) / 4.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-4, 5, (n, n)).astype(np.float64))
    U[np.diag_indices(n)] = rng.choice([-1.0, 1.0], n) * rng.integers(16, 32, n)
    return np.asfortranarray(L @ U), L, U


def _sgetrf_mixed(fmt, a, nb=0, u12=0):
    h = cdf.handle()
    h.set_param("mixed_nb", nb)
    h.set_param("lu_u12", u12)
    try:
        n = a.shape[0]
        A = cdf.to_device(a)
        W = cdf.cm_empty(n, n, torch.float32)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.full((1,), -3, dtype=torch.int32, device="cuda")
        cdf.sgetrf_mixed(fmt, A, W, ipiv, info)
        torch.cuda.synchronize()
        return cdf.to_host(W), ipiv.cpu().numpy(), int(info.item())
    finally:
        h.set_param("mixed_nb", 0)
        h.set_param("lu_u12", 0)


def _spotrf_mixed(fmt, a, nb=0):
    h = cdf.handle()
    h.set_param("mixed_nb", nb)
    try:
        n = a.shape[0]
        A = cdf.to_device(a)
        W = cdf.cm_empty(n, n, torch.float32)
        W.zero_()
        info = torch.full((1,), -3, dtype=torch.int32, device="cuda")
        cdf.spotrf_mixed(fmt, A, W, info)
        torch.cuda.synchronize()
        return cdf.to_host(W), int(info.item())
    finally:
        h.set_param("mixed_nb", 0)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("n,nb", [(40, 32), (300, 64), (300, 0), (1100, 512)])
def test_sgetrf_mixed_exact(fmt, n, nb):
    """Exactly representable factors come back exactly when U12 is formed by
    substitution.  Through an accepted L11^-1 U12 is rounded, and this L is
    very ill-conditioned across blocks, so the default path is held to the
    residual: |A - L U| <= (steps + 2) u_fmt (|L||U|) elementwise, one
    quantization of the rounded U12 per step."""
    a, L, U = _exact_lu(n, np.random.default_rng(n + nb))
    w, ipiv, info = _sgetrf_mixed(fmt, a, nb, u12=1)
    assert info == 0 and np.array_equal(ipiv, np.arange(1, n + 1))
    assert np.array_equal(np.tril(w, -1) + np.eye(n), L)
    assert np.array_equal(np.triu(w), U)
    w2, ipiv2, info2 = _sgetrf_mixed(fmt, a, nb)
    assert info2 == 0 and np.array_equal(ipiv2, ipiv)
    w2 = w2.astype(np.float64)
    L2, U2 = np.tril(w2, -1) + np.eye(n), np.triu(w2)
    bound = (n // (nb or 256) + 2) * UFMT[fmt] * (np.abs(L2) @ np.abs(U2)) + 1e-30
    r = np.abs(a - L2 @ U2)
    assert np.all(r <= bound), float(np.max(r / bound))


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("n,nb", [(40, 32), (300, 64), (300, 0), (1100, 512)])
def test_spotrf_mixed_exact(fmt, n, nb):
    rng = np.random.default_rng(7 + n)
    L = np.tril(rng.integers(-2, 3, (n, n)).astype(np.float64), -1)
    L[np.diag_indices(n)] = rng.choice([8.0, 16.0], n)
    a = np.asfortranarray(L @ L.T)
    w, info = _spotrf_mixed(fmt, a, nb)
    assert info == 0
    assert np.array_equal(np.tril(w), L)
    assert not np.any(np.triu(w, 1)), "strict upper triangle must stay untouched"


def _mixed_factor_check(w, w_or, lu_abs, fmt):
    """Two correct mixed factorizations differ by binary32 accumulation order
    (bound: (nb + 2) u32 (|L||U|)_ij per update) and, rarely, by one-code flips
    of an operand whose binary32 value sat on a rounding boundary; a flip in
    row i of L21 moves the whole row i of the trailing matrix, by at most one
    code spacing (2 u_fmt) per affected term.  Every entry must meet
    4 u_fmt (|L||U|)_ij; the typical (median) entry the accumulation bound."""
    d = np.abs(w.astype(np.float64) - w_or.astype(np.float64))
    loose = 4 * UFMT[fmt] * lu_abs + 1e-30
    assert np.all(d <= loose), float(np.max(d / loose))
    return d


@pytest.mark.parametrize("fmt", FMTS)
def test_sgetrf_mixed_vs_oracle(oracle_mod, fmt):
    n, nb = 600, 128
    a = workloads.diag_dominant(n, seed=0)
    w, ipiv, info = _sgetrf_mixed(fmt, a, nb)
    w_or, ipiv_or, info_or = oracle_mod.mixed_getrf(a, nb, oracle_mod.FMT_NAMES[fmt], 128, 128)
    assert info == info_or == 0 and np.array_equal(ipiv, ipiv_or)
    L, U = oracle_mod.split_lu(w_or.astype(np.float64))
    lu_abs = np.abs(L) @ np.abs(U)
    d = _mixed_factor_check(w, w_or, lu_abs, fmt)
    tight = (nb + 2) * U32 * lu_abs * (n // nb + 1) + 1e-30
    assert np.median(d / tight) <= 1.0


@pytest.mark.parametrize("fmt", FMTS)
def test_spotrf_mixed_vs_oracle(oracle_mod, fmt):
    n, nb = 520, 128
    a = workloads.spd_bbt(n, seed=4)
    w, info = _spotrf_mixed(fmt, a, nb)
    w_or, info_or = oracle_mod.mixed_potrf(a, nb, oracle_mod.FMT_NAMES[fmt], 128)
    assert info == info_or == 0
    L = np.tril(w_or.astype(np.float64))
    lu_abs = np.abs(L) @ np.abs(L).T
    d = _mixed_factor_check(np.tril(w), np.tril(w_or), np.tril(lu_abs), fmt)
    tight = (nb + 2) * U32 * np.tril(lu_abs) * (n // nb + 1) + 1e-30
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.median((d / tight)[low]) <= 1.0


def _solve_mixed(kind, fmt, a, b, max_iter=30):
    n = a.shape[0]
    A = cdf.to_device(a)
    B = cdf.to_device(b)
    X = cdf.cm_empty(n, b.shape[1]) if b.ndim == 2 else torch.empty(n, dtype=torch.float64, device="cuda")
    info = torch.full((1,), -3, dtype=torch.int32, device="cuda")
    fn = cdf.dgesv_mixed if kind == "lu" else cdf.dposv_mixed
    r = fn(fmt, A, B, X, info, max_iter=max_iter)
    torch.cuda.synchronize()
    r["info"] = int(info.item())
    return cdf.to_host(X), r


@pytest.mark.parametrize("fmt", ["fp64"] + FMTS)
def test_dgesv_mixed_diag_dominant(oracle_mod, fmt):
    n = 1024
    a = workloads.diag_dominant(n, seed=0)
    b = workloads.rhs_uniform(n, 1, seed=1)
    x, r = _solve_mixed("lu", fmt, a, b)
    assert r["converged"] and r["info"] == 0, r
    assert r["scaled_resid"] <= 16 and oracle_mod.hpl_scaled_residual(a, x, b) <= 16
    assert r["iters"] <= (0 if fmt == "fp64" else 10)
    lu, ipiv, _ = oracle_mod.dgetrf(a)
    x_or = oracle_mod.dgetrs(lu, ipiv, b)
    kappa = np.linalg.cond(a, np.inf)
    assert np.max(np.abs(x - x_or)) <= 2 * 16 * n * oracle_mod.EPS * kappa * np.max(np.abs(x_or))


@pytest.mark.parametrize("fmt", ["fp64"] + FMTS)
def test_dposv_mixed_spd(oracle_mod, fmt):
    n = 800
    a = workloads.spd_bbt(n, seed=11)
    b = workloads.rhs_uniform(n, 4, seed=12)
    x, r = _solve_mixed("chol", fmt, a, b)
    assert r["converged"] and r["info"] == 0, r
    assert oracle_mod.hpl_scaled_residual(a, x, b) <= 16
    l, _ = oracle_mod.dpotrf(a)
    x_or = oracle_mod.dpotrs(l, b)
    kappa = np.linalg.cond(a, np.inf)
    assert np.max(np.abs(x - x_or)) <= 2 * 16 * n * oracle_mod.EPS * kappa * np.max(np.abs(x_or))


@pytest.mark.parametrize("fmt", FMTS)
def test_dposv_mixed_kernel_matrix(oracle_mod, fmt):
    """Exponential-kernel SPD matrix (nrhs = 64), default (auto) refinement:
    every format reaches the target, E4M3 through the preconditioned-CG
    continuation (classical refinement alone needs about 28 corrections)."""
    n = 1024
    x_pts = workloads.kernel_points(n)
    a = workloads.exp_kernel_matrix(x_pts)
    b = workloads.rhs_uniform(n, 64, seed=workloads.SEED_POINTS_RHS)
    x, r = _solve_mixed("chol", fmt, a, b, max_iter=50)
    assert r["converged"], r
    assert oracle_mod.hpl_scaled_residual(a, x, b) <= 16
    l, _ = oracle_mod.dpotrf(a)
    x_or = oracle_mod.dpotrs(l, b)
    kappa = np.linalg.cond(a, np.inf)
    assert np.max(np.abs(x - x_or)) <= 2 * 16 * n * oracle_mod.EPS * kappa * np.max(np.abs(x_or))


def _solve_spd_mode(fmt, a, b, mode, max_iter=30):
    h = cdf.handle()
    h.set_param("spd_refine", mode)
    try:
        return _solve_mixed("chol", fmt, a, b, max_iter=max_iter)
    finally:
        h.set_param("spd_refine", 0)


@pytest.mark.parametrize("fmt", FMTS)
def test_dposv_mixed_shifted_pcg_density_matched(oracle_mod, fmt):
    """The full-size kernel workload's density at n = 1024 (length 0.4 for
    1024 points instead of 0.1 for 65536; kappa ~ 1e4).  E4M3's Cholesky
    breaks down, so classical refinement alone fails; the fallback (shifted
    low-precision factor, binary64 PCG) reaches the target.  Shift, number of
    factorizations and the CG iteration count follow the oracle's fallback
    (spd_solve_shifted_pcg) on the same matrix; the solution meets the HPL
    residual and the forward-error bound against the FP64 oracle solution."""
    n, nrhs = 1024, 8
    a = workloads.exp_kernel_matrix(workloads.kernel_points(n), length=0.4)
    b = workloads.rhs_uniform(n, nrhs, seed=workloads.SEED_POINTS_RHS)
    f = oracle_mod.FMT_NAMES[fmt]
    if fmt == "e4m3":
        _, r1 = _solve_spd_mode(fmt, a, b, 1)
        assert not r1["converged"] and r1["info"] > 0, r1
    x, r = _solve_spd_mode(fmt, a, b, 2)
    assert r["converged"] and r["method"] == "pcg", r
    assert oracle_mod.hpl_scaled_residual(a, x, b) <= 16
    x_o, sigma_o, nf_o, it_o, res_o, ok_o = oracle_mod.spd_solve_shifted_pcg(a, b, 256, f, 128)
    assert ok_o
    assert r["shift"] == sigma_o and r["factorizations"] == nf_o, (r, sigma_o, nf_o)
    assert abs(r["pcg_iterations"] - it_o) <= max(3, it_o // 10), (r, it_o)
    l, _ = oracle_mod.dpotrf(a)
    x_or = oracle_mod.dpotrs(l, b)
    kappa = np.linalg.cond(a, np.inf)
    assert np.max(np.abs(x - x_or)) <= 2 * 16 * n * oracle_mod.EPS * kappa * np.max(np.abs(x_or))
    # the default (auto) mode gets there too
    x2, r2 = _solve_spd_mode(fmt, a, b, 0)
    assert r2["converged"], r2
    assert oracle_mod.hpl_scaled_residual(a, x2, b) <= 16


def test_mixed_reports_non_convergence(oracle_mod):
    n = 512
    a = workloads.diag_dominant(n, seed=2)
    b = workloads.rhs_uniform(n, 1, seed=3)
    x, r = _solve_mixed("lu", "e4m3", a, b, max_iter=0)
    assert not r["converged"] and r["status"] == cdf.CDF_ERR_NOT_CONVERGED and r["iters"] == 0
    assert r["scaled_resid"] > 16
    assert abs(r["scaled_resid"] - oracle_mod.hpl_scaled_residual(a, x, b)) <= 1e-6 * r["scaled_resid"]
