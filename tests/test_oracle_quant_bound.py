"""Pins of the oracle's quantizer, I/O-bound calculator and mixed-precision
factorizations (CPU only)."""
import math

import numpy as np
import pytest
import torch

import workloads

F32_MAX = float(np.finfo(np.float32).max)


def test_decode_tables_match_library_witnesses(oracle_mod):
    # BF16: torch's bfloat16 -> float32 widening
    codes = np.arange(65536, dtype=np.uint16)
    t = torch.from_numpy(codes.view(np.int16).copy()).view(torch.bfloat16).float().numpy().astype(np.float64)
    ours = oracle_mod.decode_table(oracle_mod.FMT_BF16)
    assert np.array_equal(np.isnan(t), np.isnan(ours))
    assert np.array_equal(t[~np.isnan(t)], ours[~np.isnan(ours)])
    # FP16: numpy's IEEE binary16
    h = codes.view(np.float16).astype(np.float64)
    ours = oracle_mod.decode_table(oracle_mod.FMT_FP16)
    assert np.array_equal(np.isnan(h), np.isnan(ours))
    assert np.array_equal(h[~np.isnan(h)], ours[~np.isnan(ours)])
    # E4M3FN: torch's float8_e4m3fn
    c8 = torch.arange(256, dtype=torch.int32).to(torch.uint8).view(torch.float8_e4m3fn).float().numpy()
    ours = oracle_mod.decode_table(oracle_mod.FMT_E4M3)
    assert np.array_equal(np.isnan(c8), np.isnan(ours))
    assert np.array_equal(c8[~np.isnan(c8)].astype(np.float64), ours[~np.isnan(ours)])
    assert np.nanmax(ours) == 448.0


def _nearest_even(table, x):
    """Brute-force round to nearest over the finite decoded codes, ties to the
    code with an even last bit (the even significand)."""
    fin = np.isfinite(table)
    vals = table[fin]
    idx = np.nonzero(fin)[0]
    d = np.abs(vals - x)
    best = d.min()
    cand = idx[d == best]
    same_sign = [c for c in cand if (table[c] < 0) == (x < 0) or table[c] == 0]
    cand = same_sign or list(cand)
    even = [c for c in cand if c % 2 == 0]
    return int((even or cand)[0])


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "e4m3"])
def test_encode_is_nearest_even(oracle_mod, fmt):
    f = oracle_mod.FMT_NAMES[fmt]
    table = oracle_mod.decode_table(f)
    enc = {"bf16": oracle_mod.enc_bf16, "fp16": oracle_mod.enc_f16, "e4m3": oracle_mod.enc_e4m3}[fmt]
    rng = np.random.default_rng(1)
    top = {"bf16": 1e30, "fp16": 65000.0, "e4m3": 440.0}[fmt]
    xs = list(rng.uniform(-1, 1, 300) * np.exp(rng.uniform(-12, math.log(top), 300)))
    # exact midpoints between neighbouring positive codes (tie cases)
    fin = np.sort(table[np.isfinite(table) & (table > 0)])
    pick = rng.choice(len(fin) - 1, min(150, len(fin) - 1), replace=False)
    xs += [0.5 * (fin[i] + fin[i + 1]) for i in pick]
    xs += [-0.5 * (fin[i] + fin[i + 1]) for i in pick[:40]]
    for x in xs:
        if fmt == "bf16":
            x = float(np.float32(x))
            if 0.5 * (fin[-1] + fin[-2]) < abs(x):
                continue
        c = enc(x)
        ref = _nearest_even(table, x)
        assert table[c] == table[ref] and (c == ref or table[c] == 0), (fmt, x, c, ref)


def test_encode_matches_library_conversions(oracle_mod):
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(4000) * np.exp(rng.uniform(-8, 8, 4000))).astype(np.float32)
    bf = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert all(oracle_mod.enc_bf16(float(v)) == int(c) for v, c in zip(x, bf))
    h = x.astype(np.float16).view(np.uint16)
    xs = x.astype(np.float64)
    inr = np.abs(xs) < 65504
    assert all(oracle_mod.enc_f16(float(v)) == int(c) for v, c in zip(xs[inr], h[inr]))
    e = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    inr = np.abs(xs) < 448
    assert all(oracle_mod.enc_e4m3(float(v)) == int(c) for v, c in zip(xs[inr], e[inr]))
    # saturation instead of NaN beyond the finite range
    assert oracle_mod.enc_e4m3(1e6) == 0x7E and oracle_mod.enc_e4m3(-500.0) == 0xFE


@pytest.mark.parametrize("fmt,maxf", [("fp16", 65504.0), ("e4m3", 448.0)])
def test_tile_scale_puts_amax_in_top_binade(oracle_mod, fmt, maxf):
    f = oracle_mod.FMT_NAMES[fmt]
    rng = np.random.default_rng(3)
    amaxes = list(np.float32(np.exp(rng.uniform(-30, 30, 2000))))
    amaxes += [np.float32(maxf), np.float32(maxf / 2), np.float32(maxf * 2), np.float32(1.0),
               np.float32(np.nextafter(np.float32(maxf), np.float32(0)))]
    for a in amaxes:
        e = oracle_mod.tile_scale_exp(f, float(a))
        s = math.ldexp(float(a), e)
        assert maxf / 2 < s <= maxf, (a, e, s)
    assert oracle_mod.tile_scale_exp(f, 0.0) == 0
    assert oracle_mod.tile_scale_exp(oracle_mod.FMT_BF16, 123.0) == 0


def test_quantize_tiles(oracle_mod):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((70, 45)).astype(np.float32)
    x[:32, :16] *= 1e-3
    q, e = oracle_mod.quantize(oracle_mod.FMT_E4M3, x, 32, 16)
    assert e.shape == (3, 3)
    for ti in range(3):
        for tj in range(3):
            blk = x[ti * 32:(ti + 1) * 32, tj * 16:(tj + 1) * 16]
            assert e[ti, tj] == oracle_mod.tile_scale_exp(oracle_mod.FMT_E4M3, float(np.abs(blk).max()))
    dq = oracle_mod.dequantize(oracle_mod.FMT_E4M3, q, e, 32, 16)
    # relative error of E4M3 round-to-nearest is at most 2^-4 for normal values
    big = np.abs(x) * np.ldexp(1.0, np.repeat(np.repeat(e, 32, 0), 16, 1)[:70, :45]) >= 2 ** -6
    assert np.all(np.abs(dq - x)[big] <= 2.0 ** -4 * np.abs(x)[big])


# ---------------------------------------------------------------- I/O bound

def test_kkt_tile_volume_closed_form(oracle_mod):
    """max I J K s.t. IJ + IK + JK <= X is (X/3)^(3/2) (Sec. 6.1), by numerical
    optimisation of the normalised problem (I, J, K) = sqrt(X) (u, v, w)."""
    from scipy.optimize import minimize
    for X in (300.0, 3e4, 1e6):
        lo = 1.0 / math.sqrt(X)
        cons = {"type": "ineq", "fun": lambda v: 1.0 - (v[0] * v[1] + v[0] * v[2] + v[1] * v[2])}
        r = minimize(lambda v: -v[0] * v[1] * v[2], x0=[0.2, 0.3, 0.4], constraints=[cons],
                     bounds=[(lo, None)] * 3, method="SLSQP", options={"maxiter": 500, "ftol": 1e-15})
        best = -r.fun * X ** 1.5
        assert abs(best - oracle_mod.chi_closed_form(X)) <= 1e-6 * oracle_mod.chi_closed_form(X)
        assert np.allclose(r.x, 1 / math.sqrt(3), rtol=1e-4)


def test_intensity_minimiser_is_3m(oracle_mod):
    """argmin_X chi(X)/(X - M) = 3M and rho = sqrt(M)/2 (Sec. 6.1)."""
    from scipy.optimize import minimize_scalar
    for M in (1e2, 1e4, 20480.0):
        r = minimize_scalar(lambda X: oracle_mod.chi_closed_form(X) / (X - M),
                            bounds=(M * 1.0001, 100 * M), method="bounded",
                            options={"xatol": 1e-9 * M})
        assert abs(r.x - 3 * M) <= 1e-3 * M
        assert abs(r.fun - math.sqrt(M) / 2) <= 1e-9 * math.sqrt(M)


def test_bound_leading_terms_against_brute_force_counts(oracle_mod):
    """The bound divides the statement counts by their intensities (rho_S1 = 1,
    rho_S2 = sqrt(M)/2); brute-force counts of the loop nests agree with the
    closed forms' leading terms."""
    M = 1e4
    for N in (200, 800):
        s1 = sum(N - k - 1 for k in range(N))
        s2 = sum((N - k - 1) ** 2 for k in range(N))
        brute = s1 + s2 / (math.sqrt(M) / 2)
        assert abs(oracle_mod.io_lower_bound_elems(0, N, M) / brute - 1) < 3.0 / N
        c3 = sum((N - k - 1) * (N - k) // 2 for k in range(N))
        brute_c = N + s1 + c3 / (math.sqrt(M) / 2)
        assert abs(oracle_mod.io_lower_bound_elems(1, N, M) / brute_c - 1) < 3.0 / N
    # closed forms as printed: LU = (2N^3-6N^2+4N)/(3 sqrt M) + N(N-1)/2
    assert oracle_mod.io_lower_bound_elems(0, 10, 100) == (2000 - 600 + 40) / 30 + 45
    assert oracle_mod.io_lower_bound_elems(1, 10, 100) == 1000 / 30 + 50 + 10


# ------------------------------------------------------- mixed precision

def _exact_lu_pair(n, rng, umax):
    """A = L U with |l_ij| <= 1/2 dyadic and small-integer U: GEPP needs no
    interchanges and every intermediate is exactly representable."""
    L = np.tril(rng.integers(-2, 3, (n, n)) / 4.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-umax, umax + 1, (n, n)).astype(np.float64))
    U[np.diag_indices(n)] = rng.choice([-1.0, 1.0], n) * rng.integers(4 * umax, 8 * umax, n)
    return np.asfortranarray(L @ U), L, U


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "e4m3"])
def test_mixed_lu_exact_when_operands_are_representable(oracle_mod, fmt):
    """With operands every format holds exactly, the quantized update is exact,
    so the mixed factorization must return L and U exactly (checks signs,
    indices and the per-tile scales)."""
    rng = np.random.default_rng(5)
    n = 40
    a, L, U = _exact_lu_pair(n, rng, umax=4)
    w, ipiv, info = oracle_mod.mixed_getrf(a, nb=8, fmt=oracle_mod.FMT_NAMES[fmt], tm=16, tn=16)
    assert info == 0 and np.array_equal(ipiv, np.arange(1, n + 1))
    assert np.array_equal(np.tril(w, -1) + np.eye(n), L)
    assert np.array_equal(np.triu(w), U)


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "e4m3"])
def test_mixed_chol_exact_when_operands_are_representable(oracle_mod, fmt):
    rng = np.random.default_rng(6)
    n = 40
    L = np.tril(rng.integers(-2, 3, (n, n)).astype(np.float64), -1)
    L[np.diag_indices(n)] = rng.choice([4.0, 8.0], n)
    a = np.asfortranarray(L @ L.T)
    w, info = oracle_mod.mixed_potrf(a, nb=8, fmt=oracle_mod.FMT_NAMES[fmt], tm=16)
    assert info == 0
    assert np.array_equal(np.tril(w), L)


def test_mixed_single_panel_reduces_to_fp64_oracle(oracle_mod):
    a = workloads.lu_uniform(50, seed=8)
    w, ipiv, info = oracle_mod.mixed_getrf(a, nb=64, fmt=oracle_mod.FMT_BF16, tm=16, tn=16)
    lu, ipiv64, _ = oracle_mod.dgetrf(a.astype(np.float32).astype(np.float64))
    assert np.array_equal(ipiv, ipiv64)
    assert np.array_equal(w, lu.astype(np.float32))


@pytest.mark.parametrize("fmt,u", [("bf16", 2.0 ** -8), ("fp16", 2.0 ** -11), ("e4m3", 2.0 ** -4)])
def test_mixed_lu_backward_error_and_refinement(oracle_mod, fmt, u):
    n = 256
    a = workloads.diag_dominant(n, seed=0)
    b = workloads.rhs_uniform(n, 1, seed=1)[:, 0]
    w, ipiv, info = oracle_mod.mixed_getrf(a, nb=64, fmt=oracle_mod.FMT_NAMES[fmt], tm=32, tn=32)
    assert info == 0 and np.array_equal(ipiv, np.arange(1, n + 1))
    L, U = oracle_mod.split_lu(w.astype(np.float64))
    # backward error at the level of the update format's unit roundoff
    assert np.linalg.norm(a - L @ U) / np.linalg.norm(a) <= 4 * u
    x, it, res, ok = oracle_mod.iterative_refinement(
        a, b, lambda r: oracle_mod.solve_with_lu32(w, ipiv, r), max_iter=30)
    assert ok and res <= 16
    lu, ipiv64, _ = oracle_mod.dgetrf(a)
    x_or = oracle_mod.dgetrs(lu, ipiv64, b)
    # both solutions have scaled residual <= 16: forward error <= 2*16*n*eps*kappa_inf
    kappa = np.linalg.cond(a, np.inf)
    assert np.max(np.abs(x - x_or)) / np.max(np.abs(x_or)) <= 2 * 16 * n * oracle_mod.EPS * kappa


def test_mixed_chol_refinement(oracle_mod):
    n = 200
    a = workloads.spd_bbt(n, seed=3)
    b = workloads.rhs_uniform(n, 4, seed=4)
    w, info = oracle_mod.mixed_potrf(a, nb=64, fmt=oracle_mod.FMT_BF16, tm=32)
    assert info == 0
    x, it, res, ok = oracle_mod.iterative_refinement(
        a, b, lambda r: oracle_mod.solve_with_chol32(w, r), max_iter=30)
    assert ok and res <= 16 and it <= 10


def test_refinement_reports_non_convergence(oracle_mod):
    """A useless 'factorization' (identity) cannot converge: IR stops and says so."""
    n = 64
    a = workloads.lu_uniform(n, seed=13)
    b = workloads.rhs_uniform(n, 1, seed=14)[:, 0]
    x, it, res, ok = oracle_mod.iterative_refinement(a, b, lambda r: r.copy(), max_iter=8)
    assert not ok and res > 16
