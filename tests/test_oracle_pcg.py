"""Pins of the oracle's preconditioned conjugate gradients and of the
shifted low-precision Cholesky fallback (no GPU).

* a 2 x 2 system worked by hand in exact rationals fixes the first two CG
  iterates (the signs and the order of the alpha / beta updates);
* the exact preconditioner M = A converges in one step from x0 = 0;
* plain CG (M = I) on a matrix with three distinct eigenvalues converges in
  at most three steps (Krylov space of dimension three);
* shift_diagonal multiplies only the diagonal by (1 + sigma);
* on the exponential-kernel workload at a density matching the full-size
  one (n = 1024 points, length 0.4 instead of 0.1 for 65536 points), the E4M3
  Cholesky breaks down, and the shifted-factor PCG still reaches the HPL
  scaled residual <= 16 against the original matrix.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads


def test_cg_hand_worked_2x2(oracle_mod):
    """A = [[4,1],[1,3]], b = [1,2], x0 = 0, M = I:
    r0 = p0 = b, A p0 = [6,7], alpha0 = 5/20 = 1/4, x1 = [1/4, 1/2];
    r1 = b - alpha0 A p0 = [-1/2, 1/4], beta0 = (5/16)/5 = 1/16,
    p1 = r1 + beta0 p0 = [-7/16, 3/8], A p1 = [-11/8, 11/16],
    alpha1 = (5/16) / (55/64) = 4/11, x2 = [1/11, 7/11] = A^-1 b."""
    a = np.array([[4.0, 1.0], [1.0, 3.0]])
    b = np.array([1.0, 2.0])
    x, it, res, ok, hist = oracle_mod.pcg(a, b, lambda r: r, max_iter=5, x0=np.zeros(2), history=True)
    assert ok and it == 2
    assert np.array_equal(hist[0], np.array([0.25, 0.5]))
    want = np.array([float(Fraction(1, 11)), float(Fraction(7, 11))])
    assert np.allclose(hist[1], want, rtol=4e-16, atol=0)
    # with the preconditioner M^-1 = 2 I the iterates are the same (M is a
    # multiple of I): the preconditioned update is applied consistently
    x2, it2, _, ok2, hist2 = oracle_mod.pcg(a, b, lambda r: 2.0 * r, max_iter=5, x0=np.zeros(2), history=True)
    assert ok2 and it2 == 2 and np.array_equal(hist2[0], hist[0])


def test_pcg_exact_preconditioner_one_step(oracle_mod):
    rng = np.random.default_rng(1)
    n = 60
    g = rng.standard_normal((n, n))
    a = g @ g.T / n + np.eye(n)
    b = rng.uniform(-1, 1, (n, 3))
    x, it, res, ok = oracle_mod.pcg(a, b, lambda r: np.linalg.solve(a, r), x0=np.zeros((n, 3)))
    assert ok and it == 1 and res <= 16


def test_cg_three_distinct_eigenvalues(oracle_mod):
    rng = np.random.default_rng(2)
    n = 50
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([1.0, 3.0, 10.0], [20, 20, 10])
    a = (q * lam) @ q.T
    a = (a + a.T) / 2
    b = rng.uniform(-1, 1, n)
    x, it, res, ok = oracle_mod.pcg(a, b, lambda r: r, x0=np.zeros(n))
    assert ok and it <= 3


def test_pcg_reports_non_convergence(oracle_mod):
    rng = np.random.default_rng(3)
    n = 80
    g = rng.standard_normal((n, n))
    a = g @ g.T + 1e-3 * np.eye(n)
    b = rng.uniform(-1, 1, n)
    x, it, res, ok = oracle_mod.pcg(a, b, lambda r: r, max_iter=2, x0=np.zeros(n))
    assert not ok and it == 2 and res > 16


def test_shift_diagonal(oracle_mod):
    a = np.array([[4.0, 2.0], [2.0, 3.0]])
    s = oracle_mod.shift_diagonal(a, 0.25)
    assert np.array_equal(s, np.array([[5.0, 2.0], [2.0, 3.75]]))
    assert np.array_equal(a, np.array([[4.0, 2.0], [2.0, 3.0]]))


def test_shift_schedule(oracle_mod):
    assert oracle_mod.shift_schedule(oracle_mod.FMT_E4M3, 4) == [2.0 ** -4, 2.0 ** -2, 1.0, 4.0]
    assert oracle_mod.shift_schedule(oracle_mod.FMT_BF16, 2) == [2.0 ** -8, 2.0 ** -6]


@pytest.mark.slow
def test_shifted_pcg_recovers_e4m3_breakdown(oracle_mod):
    """Density-matched kernel matrix: E4M3 breaks down; the fallback converges."""
    n = 1024
    a = workloads.exp_kernel_matrix(workloads.kernel_points(n), length=0.4)
    b = workloads.rhs_uniform(n, 4, seed=workloads.SEED_POINTS_RHS)
    _, info = oracle_mod.mixed_potrf(a, 128, oracle_mod.FMT_E4M3, 128)
    assert info > 0
    x, sigma, nf, it, res, ok = oracle_mod.spd_solve_shifted_pcg(a, b, 128, oracle_mod.FMT_E4M3, 128)
    assert ok and sigma > 0 and nf >= 2
    assert oracle_mod.hpl_scaled_residual(a, x, b) <= 16
