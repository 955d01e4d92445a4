"""Pins of the oracle's general DAAP I/O lower bound (Sec. 3 and 4; no GPU).

* LU statement S2 (A[i,j] -= A[i,k] A[k,j]): chi(X) = (X/3)^(3/2),
  X_0 = 3M and rho = sqrt(M)/2 with tile extents sqrt(M) (Sec. 6.1);
* LU statement S1 with one out-degree-one predecessor: rho = 1 (Sec. 6.1);
* the LU program (S1 + S2) equals the printed bound
  (2N^3 - 6N^2 + 4N) / (3 sqrt(M)) + N(N-1)/2; the Cholesky program
  (three statements) equals N + N(N-1)/2 + N(N-1)(N-2)/(3 sqrt(M)), whose
  leading terms are the printed N^3/(3 sqrt(M)) + N^2/2 + N (Sec. 6.2);
* an outer product C[i,j] = a[i] b[j] (accesses a[i], b[j]): by hand,
  chi(X) = X^2/4, X_0 = 2M, rho = M;
* S2 with the access A[i,k] weighted 2 (output of a producer with rho 1/2):
  the three weighted terms are equal at the optimum, I = K = sqrt(X/6),
  J = X / (3 I), so chi(X) = I^2 J = sqrt(6) X^(3/2) / 18;
* brute force: the continuous chi(X) bounds the best integer tile from
  above and is within a small factor of it;
* Case I: two statements sharing an input array save exactly the smaller
  of their loads of it.
"""
import itertools
import math

import pytest

MM = [[0, 1], [0, 2], [2, 1]]  # S2: A[i,j], A[i,k], A[k,j] over (i, j, k)


@pytest.mark.parametrize("m", [1024.0, 4096.0, 20480.0])
def test_lu_s2_closed_form(oracle_mod, m):
    r = oracle_mod.daap_statement_bound(3, MM, [1, 1, 1], 1.0, m)
    assert r["rho"] == pytest.approx(math.sqrt(m) / 2, rel=1e-7)
    assert r["x0"] == pytest.approx(3 * m, rel=1e-4)
    for d in r["tiles"]:
        assert d == pytest.approx(math.sqrt(m), rel=1e-4)


@pytest.mark.parametrize("x", [30.0, 300.0, 3e4, 7e6])
def test_lu_s2_chi(oracle_mod, x):
    chi, _ = oracle_mod.daap_chi(3, MM, [1, 1, 1], x)
    assert chi == pytest.approx(oracle_mod.chi_closed_form(x), rel=1e-9)
    assert chi == pytest.approx((x / 3) ** 1.5, rel=1e-9)


def test_lu_s1_out_degree_one(oracle_mod):
    r = oracle_mod.daap_statement_bound(2, [[0, 1], [0]], [1, 1], 1.0, 4096.0, u=1)
    assert r["rho"] == pytest.approx(1.0, rel=1e-6)


def _lu_program(n):
    return [
        {"nvars": 2, "accesses": [[0, 1], [0]], "weights": [1, 1], "nvertices": n * (n - 1) / 2, "u": 1,
         "arrays": ["S1.A[i,k]", "S1.A[k,k]"]},
        {"nvars": 3, "accesses": MM, "weights": [1, 1, 1], "nvertices": n * (n - 1) * (n - 2) / 3, "u": 0,
         "arrays": ["S2.A[i,j]", "S2.A[i,k]", "S2.A[k,j]"]},
    ]


@pytest.mark.parametrize("n,m", [(1024.0, 4096.0), (65536.0, 20480.0)])
def test_lu_program(oracle_mod, n, m):
    q = oracle_mod.daap_program_bound(_lu_program(n), m)
    assert q == pytest.approx(oracle_mod.io_lower_bound_elems(0, n, m), rel=1e-7)
    assert q == pytest.approx((2 * n ** 3 - 6 * n ** 2 + 4 * n) / (3 * math.sqrt(m)) + n * (n - 1) / 2, rel=1e-7)


def test_cholesky_program(oracle_mod):
    n, m = 65536.0, 20480.0
    stmts = [
        {"nvars": 1, "accesses": [[0]], "weights": [1], "nvertices": n, "u": 1, "arrays": ["S1.L[k,k]"]},
        {"nvars": 2, "accesses": [[0, 1], [0]], "weights": [1, 1], "nvertices": n * (n - 1) / 2, "u": 1,
         "arrays": ["S2.L[i,k]", "S2.L[k,k]"]},
        {"nvars": 3, "accesses": MM, "weights": [1, 1, 1], "nvertices": n * (n - 1) * (n - 2) / 6, "u": 0,
         "arrays": ["S3.L[i,j]", "S3.L[i,k]", "S3.L[j,k]"]},
    ]
    q = oracle_mod.daap_program_bound(stmts, m)
    exact = n + n * (n - 1) / 2 + n * (n - 1) * (n - 2) / (3 * math.sqrt(m))
    assert q == pytest.approx(exact, rel=1e-7)
    assert q == pytest.approx(oracle_mod.io_lower_bound_elems(1, n, m), rel=1e-4)


@pytest.mark.parametrize("m", [100.0, 5000.0])
def test_outer_product(oracle_mod, m):
    r = oracle_mod.daap_statement_bound(2, [[0], [1]], [1, 1], 1.0, m)
    assert r["rho"] == pytest.approx(m, rel=1e-6)
    assert r["x0"] == pytest.approx(2 * m, rel=1e-4)
    chi, d = oracle_mod.daap_chi(2, [[0], [1]], [1, 1], 400.0)
    assert chi == pytest.approx(400.0 ** 2 / 4, rel=1e-9) and d[0] == pytest.approx(200.0, rel=1e-6)


def test_weighted_output_reuse(oracle_mod):
    for x in (60.0, 6000.0):
        chi, d = oracle_mod.daap_chi(3, MM, [1, 2, 1], x)
        assert chi == pytest.approx(math.sqrt(6) * x ** 1.5 / 18, rel=1e-8)
        i, j, k = d
        assert i == pytest.approx(math.sqrt(x / 6), rel=1e-5) and k == pytest.approx(i, rel=1e-5)


@pytest.mark.parametrize("x", [12, 40, 90])
def test_brute_force_integer_tiles(oracle_mod, x):
    best = 0
    for i, j, k in itertools.product(range(1, x + 1), repeat=3):
        if i * j + i * k + k * j <= x:
            best = max(best, i * j * k)
    chi, _ = oracle_mod.daap_chi(3, MM, [1, 1, 1], float(x))
    assert best <= chi * (1 + 1e-9) and chi <= 2.5 * best


def test_case_one_shared_input(oracle_mod):
    m = 4096.0
    s = {"nvars": 3, "accesses": MM, "weights": [1, 1, 1], "nvertices": 1e9, "u": 0}
    a = dict(s, arrays=["C1", "X", "B1"])
    b = dict(s, nvertices=2e9, arrays=["C2", "X", "B2"])
    r1 = oracle_mod.daap_statement_bound(3, MM, [1, 1, 1], 1e9, m)
    r2 = oracle_mod.daap_statement_bound(3, MM, [1, 1, 1], 2e9, m)
    loads1 = r1["access_sizes"][1] * 1e9 / r1["chi"]
    loads2 = r2["access_sizes"][1] * 2e9 / r2["chi"]
    q = oracle_mod.daap_program_bound([a, b], m)
    assert q == pytest.approx(r1["q"] + r2["q"] - min(loads1, loads2), rel=1e-9)
    c = dict(s, nvertices=2e9, arrays=["C2", "Y", "B2"])
    assert oracle_mod.daap_program_bound([a, c], m) == pytest.approx(r1["q"] + r2["q"], rel=1e-9)
