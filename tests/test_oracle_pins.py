"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test pins the oracle to something other than itself: hand-worked exact
factorizations, Leibniz determinants, exact rational elimination, textbook
special cases, invariants, and LAPACK (scipy) as an independent witness.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import workloads
from tests import golden_cases

CASES = golden_cases.load()
EPS = 2.0 ** -53


def _exact(mat):
    return golden_cases.as_f64(mat)


@pytest.mark.parametrize("name", [n for n, c in CASES.items() if c["kind"] == "lu"])
def test_lu_hand_worked_bitwise(oracle_mod, name):
    c = CASES[name]
    a = _exact(c["A"])
    lu, ipiv, info = oracle_mod.dgetrf(a)
    assert list(ipiv) == c["ipiv"]
    assert info == c["info"]
    L, U = oracle_mod.split_lu(lu)
    assert np.array_equal(L, _exact(c["L"]))
    assert np.array_equal(U, _exact(c["U"]))
    det = np.prod(np.diag(U)) * (-1) ** sum(1 for k, p in enumerate(ipiv) if p - 1 != k)
    assert det == float(c["det"])
    if "b" in c:
        b = np.array([float(v) for v in c["b"]])
        x = oracle_mod.dgetrs(lu, ipiv, b)
        assert np.array_equal(x, np.array([float(v) for v in c["x"]]))


@pytest.mark.parametrize("name", [n for n, c in CASES.items() if c["kind"] == "chol"])
def test_chol_hand_worked_bitwise(oracle_mod, name):
    c = CASES[name]
    a = _exact(c["A"])
    l, info = oracle_mod.dpotrf(a)
    assert info == c["info"]
    if info:
        return
    assert np.array_equal(np.tril(l), _exact(c["L"]))
    # the strict upper triangle is never written
    assert np.array_equal(np.triu(l, 1), np.triu(a, 1))
    assert np.prod(np.diag(l)) ** 2 == float(c["det"])
    if "b" in c:
        b = np.array([float(v) for v in c["b"]])
        x = oracle_mod.dpotrs(l, b)
        assert np.array_equal(x, np.array([float(v) for v in c["x"]]))


def test_hand_worked_fixtures_are_consistent():
    """The fixtures themselves: P A = L U and A = L L^T hold exactly in rationals."""
    for c in CASES.values():
        A = c["A"]
        n = len(A)
        if c["kind"] == "lu":
            perm = list(range(n))
            for k, p in enumerate(c["ipiv"]):
                perm[k], perm[p - 1] = perm[p - 1], perm[k]
            L, U = c["L"], c["U"]
            for i in range(n):
                for j in range(n):
                    assert sum(L[i][t] * U[t][j] for t in range(n)) == A[perm[i]][j]
        elif "L" in c:
            L = c["L"]
            for i in range(n):
                for j in range(n):
                    assert sum(L[i][t] * L[j][t] for t in range(n)) == A[i][j]


def _leibniz_det(m):
    n = len(m)
    total = Fraction(0)
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        prod = Fraction(1)
        for i in range(n):
            prod *= m[i][perm[i]]
        total += -prod if inv % 2 else prod
    return total


def _exact_gepp(m):
    """Exact rational elimination with partial pivoting; also reports the
    smallest relative gap between the chosen pivot and any other candidate."""
    n = len(m)
    a = [[Fraction(x) for x in r] for r in m]
    ipiv, gap = [], float("inf")
    for k in range(n):
        col = [abs(a[i][k]) for i in range(k, n)]
        p = k + max(range(len(col)), key=lambda t: (col[t], -t))
        best = abs(a[p][k])
        others = [abs(a[i][k]) for i in range(k, n) if i != p]
        if best > 0 and others:
            gap = min(gap, float((best - max(others)) / best))
        ipiv.append(p + 1)
        if a[p][k] == 0:
            continue
        a[k], a[p] = a[p], a[k]
        for i in range(k + 1, n):
            a[i][k] /= a[k][k]
            for j in range(k + 1, n):
                a[i][j] -= a[i][k] * a[k][j]
    return a, ipiv, gap


def test_det_matches_leibniz_brute_force(oracle_mod):
    rng = np.random.default_rng(11)
    for n in range(1, 8):
        for _ in range(6):
            m = rng.integers(-9, 10, size=(n, n))
            a = np.asfortranarray(m.astype(np.float64))
            lu, ipiv, info = oracle_mod.dgetrf(a)
            swaps = sum(1 for k, p in enumerate(ipiv) if p - 1 != k)
            det = float(np.prod(np.diag(lu))) * (-1) ** swaps
            ref = _leibniz_det([[Fraction(int(v)) for v in r] for r in m])
            assert abs(det - float(ref)) <= 1e-9 * max(1.0, abs(float(ref)))
            assert (info != 0) == (ref == 0) or abs(float(ref)) < 1e-6


def test_pivots_match_exact_rational_gepp(oracle_mod):
    rng = np.random.default_rng(12)
    checked = 0
    for trial in range(200):
        n = int(rng.integers(2, 9))
        m = rng.integers(-20, 21, size=(n, n))
        exact, ipiv_ex, gap = _exact_gepp([[int(v) for v in r] for r in m])
        if gap < 1e-9:
            continue  # an exact (or rounding-level) tie: pinned separately by LU3
        lu, ipiv, info = oracle_mod.dgetrf(np.asfortranarray(m.astype(np.float64)))
        assert list(ipiv) == ipiv_ex
        ref = np.array([[float(x) for x in r] for r in exact])
        assert np.allclose(lu, ref, rtol=1e-12, atol=1e-12)
        checked += 1
    assert checked >= 100


def test_special_cases(oracle_mod):
    # n = 1
    lu, ipiv, info = oracle_mod.dgetrf(np.array([[3.0]], order="F"))
    assert lu[0, 0] == 3.0 and list(ipiv) == [1] and info == 0
    # permutation matrix: GEPP undoes it with L = U = I
    rng = np.random.default_rng(3)
    perm = rng.permutation(16)
    a = np.asfortranarray(np.eye(16)[perm])
    lu, ipiv, info = oracle_mod.dgetrf(a)
    assert np.array_equal(lu, np.eye(16)) and info == 0
    assert np.array_equal(a[oracle_mod.ipiv_to_perm(ipiv, 16)], np.eye(16))
    # upper triangular input: no interchanges, L = I, U = A
    u = np.asfortranarray(np.triu(rng.uniform(1, 2, (12, 12))))
    lu, ipiv, info = oracle_mod.dgetrf(u)
    assert list(ipiv) == list(range(1, 13)) and np.array_equal(lu, u)
    # zero matrix: info = 1, nothing changes
    z = np.zeros((5, 5), order="F")
    lu, ipiv, info = oracle_mod.dgetrf(z)
    assert info == 1 and np.array_equal(lu, z) and list(ipiv) == [1, 2, 3, 4, 5]
    # diagonal SPD: Cholesky factor is the elementwise square root
    d = np.diag([4.0, 9.0, 16.0, 0.25])
    l, info = oracle_mod.dpotrf(np.asfortranarray(d))
    assert info == 0 and np.array_equal(np.diag(l), [2.0, 3.0, 4.0, 0.5])


@pytest.mark.parametrize("n", [1, 2, 7, 64, 255, 600])
def test_lu_invariants_random(oracle_mod, n):
    a = workloads.lu_uniform(n, seed=100 + n)
    lu, ipiv, info = oracle_mod.dgetrf(a)
    assert info == 0
    L, U = oracle_mod.split_lu(lu)
    assert np.all(np.abs(np.tril(lu, -1)) <= 1.0)
    assert oracle_mod.lu_backward_error(a, lu, ipiv) <= 10.0
    assert np.all(ipiv >= np.arange(1, n + 1))


@pytest.mark.parametrize("n", [1, 3, 64, 300])
def test_chol_invariants_random(oracle_mod, n):
    a = workloads.spd_bbt(n, seed=200 + n)
    l, info = oracle_mod.dpotrf(a)
    assert info == 0
    assert np.all(np.diag(l) > 0)
    assert oracle_mod.chol_backward_error(a, l) <= 10.0


@pytest.mark.parametrize("n", [64, 256, 1024])
def test_pivots_match_lapack_witness(oracle_mod, n):
    """LAPACK's blocked dgetrf (scipy) picks the same pivots despite a
    different summation order (premise of the identical-pivot requirement)."""
    from scipy.linalg import lu_factor
    a = workloads.lu_uniform(n, seed=300 + n)
    lu, ipiv, info = oracle_mod.dgetrf(a)
    lu_ref, piv_ref = lu_factor(a)
    assert np.array_equal(ipiv, piv_ref + 1)
    assert np.allclose(lu, lu_ref, rtol=0, atol=1e-10 * n)


def test_cholesky_matches_numpy_witness(oracle_mod):
    n = 200
    a = workloads.spd_bbt(n, seed=7)
    l, info = oracle_mod.dpotrf(a)
    ref = np.linalg.cholesky(a)
    # kappa(A) <= ~5 for B B^T / n + I, so the factors agree to a few n * eps
    assert np.max(np.abs(np.tril(l) - ref)) <= 50 * n * EPS * np.max(np.abs(ref))


def test_bitwise_independent_of_threads(oracle_mod):
    a = workloads.lu_uniform(300, seed=5)
    s = workloads.spd_bbt(300, seed=6)
    old = oracle_mod.get_threads()
    try:
        oracle_mod.set_threads(1)
        r1 = oracle_mod.dgetrf(a)
        c1 = oracle_mod.dpotrf(s)
        oracle_mod.set_threads(max(2, old))
        r8 = oracle_mod.dgetrf(a)
        c8 = oracle_mod.dpotrf(s)
    finally:
        oracle_mod.set_threads(old)
    assert np.array_equal(r1[0], r8[0]) and np.array_equal(r1[1], r8[1])
    assert np.array_equal(c1[0], c8[0])


def test_partial_steps_leave_schur_complement(oracle_mod):
    n, s = 80, 17
    a = workloads.lu_uniform(n, seed=9)
    full, ipiv_full, _ = oracle_mod.dgetrf(a)
    part, ipiv_part, _ = oracle_mod.dgetrf(a, ksteps=s)
    assert np.array_equal(ipiv_part[:s], ipiv_full[:s])
    # P A = [L11 0; L21 I] [U11 U12; 0 S]
    p = oracle_mod.ipiv_to_perm(np.concatenate([ipiv_part[:s], np.arange(s + 1, n + 1)]), n)
    Lb = np.eye(n)
    Lb[:, :s] = np.tril(part[:, :s], -1) + np.eye(n)[:, :s]
    Ub = np.triu(part)
    Ub[s:, s:] = part[s:, s:]
    assert np.max(np.abs(a[p] - Lb @ Ub)) <= 1e-13 * n
    # finishing the Schur complement reproduces the full factorization's pivots
    rest, ipiv_rest, _ = oracle_mod.dgetrf(part[s:, s:])
    assert np.array_equal(ipiv_rest + s, ipiv_full[s:])
    # Cholesky: partial steps leave the Schur complement in the trailing block
    c = workloads.spd_bbt(n, seed=10)
    lfull, _ = oracle_mod.dpotrf(c)
    lpart, _ = oracle_mod.dpotrf(c, ksteps=s)
    assert np.allclose(np.tril(lpart[:, :s]), np.tril(lfull[:, :s]), rtol=0, atol=0)
    lrest, _ = oracle_mod.dpotrf(lpart[s:, s:])
    assert np.max(np.abs(np.tril(lrest) - np.tril(lfull[s:, s:]))) <= 1e-13


def test_getrs_potrs_residual(oracle_mod):
    n = 200
    a = workloads.lu_uniform(n, seed=21)
    b = workloads.rhs_uniform(n, 3, seed=22)
    lu, ipiv, _ = oracle_mod.dgetrf(a)
    x = oracle_mod.dgetrs(lu, ipiv, b)
    assert oracle_mod.hpl_scaled_residual(a, x, b) <= 16
    assert np.allclose(x, np.linalg.solve(a, b), rtol=1e-9, atol=1e-9)
    s = workloads.spd_bbt(n, seed=23)
    l, _ = oracle_mod.dpotrf(s)
    xs = oracle_mod.dpotrs(l, b)
    assert oracle_mod.hpl_scaled_residual(s, xs, b) <= 16
    assert np.allclose(xs, np.linalg.solve(s, b), rtol=1e-10, atol=1e-12)


def test_diag_dominant_needs_no_interchanges(oracle_mod):
    a = workloads.diag_dominant(300, seed=0)
    _, ipiv, info = oracle_mod.dgetrf(a)
    assert info == 0 and np.array_equal(ipiv, np.arange(1, 301))
