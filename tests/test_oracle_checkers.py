"""Pins of the oracle's acceptance checkers (no GPU).

Every correctness claim rests on four functions of ``oracle``: the HPL
scaled residual, the LU and Cholesky scaled backward errors, and the exact
flop counts of the first elimination steps.  Each is checked here against a
value worked out by hand (exact rationals, then one rounding), so that a slip
in eps (2^-52 for 2^-53), in the norm (1 or 2 for inf / Frobenius), in the
factor n, or in a term left out fails a test.  The hand-worked inputs are the
LU3 and CH3 fixtures of tests/golden/hand_worked.txt, whose exact factors
are pinned in test_oracle_pins.py.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from tests import golden_cases

EPS = Fraction(1, 2 ** 53)
CASES = golden_cases.load()
DELTA = 2.0 ** -40  # a perturbation whose products with the fixture entries are exact


def _close(got, want, rel=1e-13):
    return abs(got - float(want)) <= rel * abs(float(want))


def test_eps_is_unit_roundoff(oracle_mod):
    assert oracle_mod.EPS == 2.0 ** -53


# ------------------------------------------------------ HPL scaled residual

def test_hpl_residual_hand_worked_lu3(oracle_mod):
    """LU3: A = [[2,1,1],[4,-6,0],[-2,7,2]], b = [5,-2,9], exact x = [1,1,2].
    x~ = [1, 1, 2 + d]: A x~ - b = d * A[:, 2] = [d, 0, 2d], so
    ||r||_inf = 2d; ||A||_inf = max row sum = max(4, 10, 11) = 11 (the max
    column sum would be 14); ||x~||_inf = 2 + d; ||b||_inf = 9; n = 3.
    scaled = 2d / (eps (11 (2 + d) + 9) 3)."""
    c = CASES["LU3"]
    a = golden_cases.as_f64(c["A"])
    b = np.array([float(v) for v in c["b"]])
    d = Fraction(DELTA)
    x = np.array([1.0, 1.0, 2.0 + DELTA])
    want = 2 * d / (EPS * (11 * (2 + d) + 9) * 3)
    assert _close(oracle_mod.hpl_scaled_residual(a, x, b), want)
    # the exact solution has residual exactly zero
    assert oracle_mod.hpl_scaled_residual(a, np.array([1.0, 1.0, 2.0]), b) == 0.0


def test_hpl_residual_max_over_columns(oracle_mod):
    """Two right-hand sides, each with its own ||x|| and ||b||: the result is
    the larger of the two per-column values (not a norm over the block)."""
    c = CASES["LU3"]
    a = golden_cases.as_f64(c["A"])
    x_exact = np.array([1.0, 1.0, 2.0])
    b1 = a @ x_exact                          # [5, -2, 9]
    x2_exact = np.array([2.0, 0.0, 0.0])
    b2 = a @ x2_exact                         # [4, 8, -4]
    x1 = np.array([1.0, 1.0, 2.0 + DELTA])    # r1 = [d, 0, 2d]
    x2 = np.array([2.0 + DELTA, 0.0, 0.0])    # r2 = d * A[:, 0] = [2d, 4d, -2d]
    d = Fraction(DELTA)
    col1 = 2 * d / (EPS * (11 * (2 + d) + 9) * 3)
    col2 = 4 * d / (EPS * (11 * (2 + d) + 8) * 3)
    got = oracle_mod.hpl_scaled_residual(a, np.stack([x1, x2], 1), np.stack([b1, b2], 1))
    assert _close(got, max(col1, col2))
    assert col2 > col1


# ---------------------------------------------------------- backward errors

def test_lu_backward_error_hand_worked_lu3(oracle_mod):
    """LU3's exact factors with ipiv = [2, 2, 3] (P swaps rows 0 and 1).
    U(2,2) += d: P A - L U' = -d L[:, 2] e_2^T = -d e_2 e_2^T, Frobenius d.
    ||A||_F^2 = 4+1+1+16+36+0+4+49+4 = 115, n = 3:
    error = d / (sqrt(115) 3 eps)."""
    c = CASES["LU3"]
    a = golden_cases.as_f64(c["A"])
    L = golden_cases.as_f64(c["L"])
    U = golden_cases.as_f64(c["U"])
    ipiv = np.array(c["ipiv"], dtype=np.int32)
    lu = np.tril(L, -1) + U
    assert oracle_mod.lu_backward_error(a, lu, ipiv) == 0.0
    lu2 = lu.copy()
    lu2[2, 2] += DELTA
    want = DELTA / (math.sqrt(115.0) * 3 * 2.0 ** -53)
    assert _close(oracle_mod.lu_backward_error(a, lu2, ipiv), want, 1e-12)


def test_lu_backward_error_multiplier_row_and_permutation(oracle_mod):
    """L(2,0) += d adds d * U[0, :] = d [4, -6, 0] to row 2 of L U:
    Frobenius d sqrt(52).  The same factors read with the identity
    permutation (ignoring ipiv) leave rows 0 and 1 of A swapped: a large
    error, so a checker that ignored ipiv would fail the first value."""
    c = CASES["LU3"]
    a = golden_cases.as_f64(c["A"])
    L = golden_cases.as_f64(c["L"])
    U = golden_cases.as_f64(c["U"])
    ipiv = np.array(c["ipiv"], dtype=np.int32)
    lu = np.tril(L, -1) + U
    lu[2, 0] += DELTA
    want = DELTA * math.sqrt(52.0) / (math.sqrt(115.0) * 3 * 2.0 ** -53)
    assert _close(oracle_mod.lu_backward_error(a, lu, ipiv), want, 1e-12)
    lu[2, 0] -= DELTA
    # rows 0 and 1 of A differ by [-2, 7, 1]: ||.||_F of the two-row
    # difference = sqrt(2 * (4 + 49 + 1))
    want_id = math.sqrt(2 * 54.0) / (math.sqrt(115.0) * 3 * 2.0 ** -53)
    assert _close(oracle_mod.lu_backward_error(a, lu, np.array([1, 2, 3], dtype=np.int32)), want_id, 1e-12)


def test_chol_backward_error_hand_worked_ch3(oracle_mod):
    """CH3: A = [[4,2,-2],[2,10,2],[-2,2,6]], L = [[2,0,0],[1,3,0],[-1,1,2]].
    L(2,2) += d: (L + D)(L + D)^T - L L^T has one nonzero, (2,2) =
    2 * 2d + d^2.  ||A||_F^2 = 16+4+4+4+100+4+4+4+36 = 176, n = 3."""
    c = CASES["CH3"]
    a = golden_cases.as_f64(c["A"])
    L = golden_cases.as_f64(c["L"])
    assert oracle_mod.chol_backward_error(a, L) == 0.0
    L2 = L.copy()
    L2[2, 2] += DELTA
    want = (4 * DELTA + DELTA ** 2) / (math.sqrt(176.0) * 3 * 2.0 ** -53)
    assert _close(oracle_mod.chol_backward_error(a, L2), want, 1e-12)


def test_chol_backward_error_off_diagonal_and_lower_only(oracle_mod):
    """L(2,0) += d: the change of L L^T is d (L[:,0] e_2^T + e_2 L[:,0]^T)
    + d^2 e_2 e_2^T with L[:,0] = [2, 1, -1]: entries (0,2), (2,0) = 2d,
    (1,2), (2,1) = d, (2,2) = -2d + d^2.  Frobenius^2 = 2(4d^2) + 2 d^2 +
    (2d - d^2)^2.  Garbage in the strict upper triangles of A and of the
    factor changes nothing: only lower triangles are read."""
    c = CASES["CH3"]
    a = golden_cases.as_f64(c["A"])
    L = golden_cases.as_f64(c["L"])
    L2 = L.copy()
    L2[2, 0] += DELTA
    fro = math.sqrt(10 * DELTA ** 2 + (2 * DELTA - DELTA ** 2) ** 2)
    want = fro / (math.sqrt(176.0) * 3 * 2.0 ** -53)
    assert _close(oracle_mod.chol_backward_error(a, L2), want, 1e-12)
    a_up = a.copy()
    a_up[0, 1], a_up[0, 2], a_up[1, 2] = 1e300, -7.0, np.nan
    L2[0, 1], L2[1, 2] = 5.0, -3.0
    assert _close(oracle_mod.chol_backward_error(a_up, L2), want, 1e-12)


# ---------------------------------------------------------- flop counts

def _count_lu_ops(n, steps):
    """Operations of unblocked elimination counted one by one: one division
    per multiplier, one multiply and one subtract per trailing entry."""
    ops = 0
    for k in range(min(n, steps)):
        for i in range(k + 1, n):
            ops += 1
            for j in range(k + 1, n):
                ops += 2
    return ops


def _count_chol_ops(n, steps):
    """Cholesky listing, lower: one square root, one division per entry of
    the column below it, one multiply and one subtract per updated entry of
    the lower trailing triangle (j in k+1..n-1, i in j..n-1)."""
    ops = 0
    for k in range(min(n, steps)):
        ops += 1
        ops += n - k - 1
        for j in range(k + 1, n):
            for i in range(j, n):
                ops += 2
    return ops


def test_step_flops_n2_exact(oracle_mod):
    # 2N^3/3 - N^2/2 - N/6 = 3 and N^3/3 + N^2/2 + N/6 = 5 at N = 2
    assert oracle_mod.lu_step_flops(2, 2) == 3
    assert oracle_mod.chol_step_flops(2, 2) == 5


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 40])
def test_step_flops_closed_forms(oracle_mod, n):
    lu = Fraction(2 * n ** 3, 3) - Fraction(n ** 2, 2) - Fraction(n, 6)
    ch = Fraction(n ** 3, 3) + Fraction(n ** 2, 2) + Fraction(n, 6)
    assert oracle_mod.lu_step_flops(n, n) == lu
    assert oracle_mod.chol_step_flops(n, n) == ch


@pytest.mark.parametrize("n,steps", [(7, 0), (7, 1), (7, 3), (9, 9), (12, 5), (30, 17), (6, 50)])
def test_step_flops_brute_force(oracle_mod, n, steps):
    assert oracle_mod.lu_step_flops(n, steps) == _count_lu_ops(n, steps)
    assert oracle_mod.chol_step_flops(n, steps) == _count_chol_ops(n, steps)


def test_flop_conventions(oracle_mod):
    assert oracle_mod.lu_flops(3) == 18.0 and oracle_mod.chol_flops(3) == 9.0
