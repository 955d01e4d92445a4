"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np

EPS = 2.0 ** -53


def lu_parity_tolerance(lu_or: np.ndarray) -> np.ndarray:
    """Elementwise bound for two correct FP64 LU factorizations that differ only
    in rounding order: 16 n eps (|L||U|)_ij, divided by |u_jj| for L entries
    (they are quotients by the pivot)."""
    n = lu_or.shape[0]
    L = np.tril(lu_or, -1) + np.eye(n)
    U = np.triu(lu_or)
    LU = np.abs(L) @ np.abs(U)
    tol = 16 * n * EPS * LU
    d = np.abs(np.diag(U))
    d[d == 0] = 1.0
    low = np.tril(np.ones((n, n), dtype=bool), -1)
    tol[low] = (tol / d[None, :])[low]
    return tol + 1e-300


def chol_parity_tolerance(l_or: np.ndarray) -> np.ndarray:
    n = l_or.shape[0]
    L = np.tril(l_or)
    LL = np.abs(L) @ np.abs(L).T
    d = np.abs(np.diag(L))
    return np.tril(16 * n * EPS * LL / d[None, :]) + 1e-300


def first_pivot_mismatch(ip_gpu, ip_or, a, oracle):
    """Describe the first differing pivot: step, candidates and their gap."""
    k = int(np.nonzero(np.asarray(ip_gpu) != np.asarray(ip_or))[0][0])
    part, _, _ = oracle.dgetrf(a, ksteps=k)
    col = np.abs(part[k:, k])
    g, o = int(ip_gpu[k]) - 1 - k, int(ip_or[k]) - 1 - k
    gap = abs(col[o] - col[g]) / max(col[o], 1e-300)
    return f"step {k}: gpu row {g + k} |a|={col[g]!r}, oracle row {o + k} |a|={col[o]!r}, rel gap {gap:.3e}"
