"""Tournament pivoting on the GPU (Sec. 7.3) against the oracle.

* FP64 LU with tournament leaves: pivots identical to the oracle's CALU
  factorization (tournament_pivots on each 32-column leaf) for several
  block sizes and fan-ins (one to five rounds), factors to rounding;
* one block per leaf: the pivots of LU with partial pivoting;
* the mixed-precision LU with tournament leaves: on exactly representable
  factors behind a row permutation, W and the pivots equal the oracle's bit
  for bit; on the refinement workload with shuffled rows the refined solve
  reaches the HPL residual;
* a zero column: info names it as the oracle does.
"""
import numpy as np
import pytest
import torch

import paper_2108_09337_amd as cdf
import workloads

pytestmark = pytest.mark.gpu


def _params(block, fanin, pivot=1):
    h = cdf.handle()
    h.set_param("lu_pivot", pivot)
    h.set_param("tourn_block", block)
    h.set_param("tourn_fanin", fanin)
    return h


def _reset():
    _params(0, 0, 0)


def _getrf(a):
    n = a.shape[0]
    A = cdf.to_device(a)
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    info = torch.full((1,), -3, dtype=torch.int32, device="cuda")
    cdf.dgetrf(A, ipiv, info)
    torch.cuda.synchronize()
    return cdf.to_host(A), ipiv.cpu().numpy(), int(info.item())


@pytest.mark.parametrize("n,block,fanin", [(600, 256, 8), (600, 32, 2), (777, 64, 3), (2100, 256, 8), (1500, 128, 2)])
def test_getrf_tournament_vs_oracle(oracle_mod, n, block, fanin):
    a = workloads.lu_uniform(n, seed=n + block)
    print(f"tournament getrf n={n} block={block} fanin={fanin}", flush=True)
    try:
        _params(block, fanin)
        lu, ipiv, info = _getrf(a)
    finally:
        _reset()
    lu_or, ipiv_or, info_or = oracle_mod.calu_panel(a, 32, block, fanin)
    assert info == info_or == 0
    assert np.array_equal(ipiv, ipiv_or)
    L, U = oracle_mod.split_lu(lu_or)
    scale = np.abs(L) @ np.abs(U)
    d = np.abs(lu - lu_or)
    assert np.all(d <= 64 * n * oracle_mod.EPS * scale + 1e-300), float(np.max(d / (n * oracle_mod.EPS * scale)))
    _, gp, _ = oracle_mod.dgetrf(a)
    assert not np.array_equal(ipiv, gp)  # several blocks: not the partial-pivoting order
    assert oracle_mod.lu_backward_error(a, lu, ipiv) <= 16


def test_getrf_tournament_one_block_is_partial_pivoting(oracle_mod):
    n = 250
    a = workloads.lu_uniform(n, seed=5)
    try:
        _params(256, 8)
        lu, ipiv, info = _getrf(a)
    finally:
        _reset()
    lu_or, ipiv_or, _ = oracle_mod.dgetrf(a)
    assert info == 0 and np.array_equal(ipiv, ipiv_or)
    assert np.max(np.abs(lu - lu_or)) <= 1e-12


def test_getrf_tournament_zero_column_info(oracle_mod):
    n = 300
    a = workloads.lu_uniform(n, seed=9)
    a[:, 70] = 0.0
    try:
        _params(64, 2)
        lu, ipiv, info = _getrf(a)
    finally:
        _reset()
    _, ipiv_or, info_or = oracle_mod.calu_panel(a, 32, 64, 2)
    assert info == info_or == 71
    assert np.array_equal(ipiv[:70], ipiv_or[:70])


def _permuted_exact_lu(n, rng):
    """Rows of L U shuffled, with |L| <= 1/32 off the diagonal and |U_jj| >= 16:
    every local LU of the tournament works on dyadic values (exact in both
    implementations), and the rows of the permutation stay each column's
    dominant candidates, so the final pivots recover it and the factors stay
    exact through the low-precision updates."""
    L = np.tril(rng.integers(-2, 3, (n, n)) / 64.0, -1) + np.eye(n)
    U = np.triu(rng.integers(-4, 5, (n, n)).astype(np.float64))
    U[np.diag_indices(n)] = rng.choice([-1.0, 1.0], n) * rng.integers(16, 32, n)
    perm = rng.permutation(n)
    return np.asfortranarray((L @ U)[perm])


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_mixed_tournament_exact(oracle_mod, fmt):
    n, nb, block, fanin = 300, 64, 32, 2
    a = _permuted_exact_lu(n, np.random.default_rng(17))
    h = _params(block, fanin)
    h.set_param("mixed_nb", nb)
    h.set_param("lu_u12", 1)
    try:
        A = cdf.to_device(a)
        W = cdf.cm_empty(n, n, torch.float32)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.full((1,), -3, dtype=torch.int32, device="cuda")
        cdf.sgetrf_mixed(fmt, A, W, ipiv, info)
        torch.cuda.synchronize()
        w, piv, inf = cdf.to_host(W), ipiv.cpu().numpy(), int(info.item())
    finally:
        h.set_param("mixed_nb", 0)
        h.set_param("lu_u12", 0)
        _reset()
    w_or, piv_or, inf_or = oracle_mod.mixed_getrf(a, nb, oracle_mod.FMT_NAMES[fmt], 128, 128,
                                                  tournament=(32, block, fanin))
    assert inf == inf_or == 0
    assert np.array_equal(piv, piv_or)
    assert np.array_equal(w, w_or)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_dgesv_mixed_tournament_converges(oracle_mod, fmt):
    """The refinement workload (row diagonally dominant) with its rows
    shuffled, so that every panel interchanges rows."""
    n = 2048
    a = np.asfortranarray(workloads.diag_dominant(n, seed=21)[np.random.default_rng(21).permutation(n)])
    b = workloads.rhs_uniform(n, 1, seed=22)
    try:
        _params(256, 8)
        A = cdf.to_device(a)
        B = cdf.to_device(b)
        X = cdf.cm_empty(n, 1)
        info = torch.full((1,), -3, dtype=torch.int32, device="cuda")
        r = cdf.dgesv_mixed(fmt, A, B, X, info, max_iter=30)
        torch.cuda.synchronize()
        x = cdf.to_host(X)
    finally:
        _reset()
    assert r["converged"] and int(info.item()) == 0, r
    assert r["iters"] <= 10
    assert oracle_mod.hpl_scaled_residual(a, x, b) <= 16
