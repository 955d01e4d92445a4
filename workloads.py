"""Seeded synthetic inputs for the dense LU / Cholesky workloads.

This module is shared by the tests, the benchmark and the oracle's callers.
It holds no arithmetic of the factorization method itself: it only draws
matrices and right-hand sides with the distributions the workloads name.

All matrices are returned as numpy float64 arrays in column-major (Fortran)
order, i.e. element (i, j) of an n x n matrix sits at offset i + j * n.

Seeds follow one convention everywhere:
  seed 0 -> matrix entries, seed 1 -> right-hand sides,
  seed 2 -> kernel-matrix points, seed 3 -> kernel-matrix right-hand sides,
  seed 4 -> batched problem sizes.
"""
from __future__ import annotations

import hashlib

import numpy as np

SEED_MATRIX = 0
SEED_RHS = 1
SEED_POINTS = 2
SEED_POINTS_RHS = 3
SEED_BATCH = 4


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def lu_uniform(n: int, seed: int = SEED_MATRIX, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """General matrix with iid uniform[lo, hi) entries (column-major)."""
    a = _rng(seed).uniform(lo, hi, size=(n, n))
    return np.asfortranarray(a)


def rhs_uniform(n: int, nrhs: int = 1, seed: int = SEED_RHS) -> np.ndarray:
    """Right-hand sides with iid uniform[-1, 1) entries, shape (n, nrhs), column-major."""
    return np.asfortranarray(_rng(seed).uniform(-1.0, 1.0, size=(n, nrhs)))


def spd_bbt(n: int, seed: int = SEED_MATRIX) -> np.ndarray:
    """SPD matrix A = B B^T / n + I with B iid N(0, 1) (column-major).

    The product is symmetrised bit-exactly (lower triangle mirrored) so that the
    oracle and the device path see the same bits whichever triangle they read.
    """
    b = _rng(seed).standard_normal(size=(n, n))
    a = (b @ b.T) / n
    a[np.diag_indices(n)] += 1.0
    a = np.tril(a) + np.tril(a, -1).T
    return np.asfortranarray(a)


def diag_dominant(n: int, seed: int = SEED_MATRIX) -> np.ndarray:
    """Entries iid uniform[-0.5, 0.5); then a_ii := sum_j |a_ij| over the full drawn row.

    The row sum includes the original diagonal draw, so the matrix is strictly
    row diagonally dominant almost surely.
    """
    a = _rng(seed).uniform(-0.5, 0.5, size=(n, n))
    a[np.diag_indices(n)] = np.abs(a).sum(axis=1)
    return np.asfortranarray(a)


def kernel_points(n: int, seed: int = SEED_POINTS) -> np.ndarray:
    """n points iid uniform in the unit cube [0, 1]^3, shape (n, 3)."""
    return _rng(seed).uniform(0.0, 1.0, size=(n, 3))


def exp_kernel_matrix(x: np.ndarray, length: float = 0.1, nugget: float = 1e-2) -> np.ndarray:
    """K_ij = exp(-||x_i - x_j||_2 / length) + nugget * delta_ij, column-major float64."""
    n = x.shape[0]
    k = np.empty((n, n), dtype=np.float64, order="F")
    step = 2048
    for j0 in range(0, n, step):
        j1 = min(n, j0 + step)
        d = x[:, None, :] - x[None, j0:j1, :]
        k[:, j0:j1] = np.exp(-np.sqrt((d * d).sum(axis=2)) / length)
    k[np.diag_indices(n)] += nugget
    return k


def batch_sizes(count: int = 4096, lo: int = 16, hi: int = 512, seed: int = SEED_BATCH) -> np.ndarray:
    """Problem sizes N_i = round(exp(U[ln lo, ln hi])) as int32."""
    u = _rng(seed).uniform(np.log(lo), np.log(hi), size=count)
    return np.rint(np.exp(u)).astype(np.int32)


def batch_kinds(count: int) -> np.ndarray:
    """Problem kinds: 0 (LU) for even i, 1 (Cholesky) for odd i."""
    return (np.arange(count) % 2).astype(np.int32)


def batch_problem(i: int, n: int, kind: int, seed: int = SEED_MATRIX) -> np.ndarray:
    """Matrix of batched problem i: LU -> uniform[-1,1], Cholesky -> B B^T / n + I."""
    s = 1_000_003 * (seed + 1) + i
    return lu_uniform(n, seed=s) if kind == 0 else spd_bbt(n, seed=s)


def diag_dominant_torch(n: int, seed: int = SEED_MATRIX, device: str = "cuda"):
    """diag_dominant() drawn on the GPU with torch's seeded generator (same
    distribution, different stream), column-major view; for sizes where a
    host draw would dominate the run time."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    a = torch.empty((n, n), dtype=torch.float64, device=device)  # a[j, i] = entry (i, j)
    a.uniform_(-0.5, 0.5, generator=g)
    rows = torch.zeros(n, dtype=torch.float64, device=device)
    for j0 in range(0, n, 2048):        # row sums of the column-major matrix, in column slabs
        rows += a[j0:j0 + 2048].abs().sum(dim=0)
    a.diagonal().copy_(rows)
    return a.t()


def lu_uniform_torch(n: int, seed: int = SEED_MATRIX, device: str = "cuda"):
    """lu_uniform() drawn on the GPU with torch's seeded generator (same
    distribution, different stream), as a column-major view."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    a = torch.empty((n, n), dtype=torch.float64, device=device)  # a[j, i] = entry (i, j)
    a.uniform_(-1.0, 1.0, generator=g)
    return a.t()


def spd_bbt_torch(n: int, seed: int = SEED_MATRIX, device: str = "cuda"):
    """spd_bbt() drawn on the GPU: B B^T / n + I with B iid N(0, 1) from
    torch's seeded generator, as a column-major view.  The product is
    symmetric up to rounding; Cholesky reads its lower triangle only."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    b = torch.empty((n, n), dtype=torch.float64, device=device)
    b.normal_(0.0, 1.0, generator=g)
    s = torch.mm(b, b.t().contiguous())
    del b
    s.div_(n)
    s.diagonal().add_(1.0)
    torch.cuda.empty_cache()
    return s.t()


def exp_kernel_matrix_torch(x: np.ndarray, length: float = 0.1, nugget: float = 1e-2, device: str = "cuda"):
    """exp_kernel_matrix() evaluated on the GPU (same points, same formula:
    differences, squares, sum, sqrt, exp), as a column-major view."""
    import torch
    n = x.shape[0]
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=torch.float64)
    k = torch.empty((n, n), dtype=torch.float64, device=device)  # k[j, i] = entry (i, j); K is symmetric
    step = 1024
    for j0 in range(0, n, step):
        j1 = min(n, j0 + step)
        d = xt[j0:j1, None, :] - xt[None, :, :]
        k[j0:j1] = torch.exp(-torch.sqrt((d * d).sum(dim=2)) / length)
        del d
    k.diagonal().add_(nugget)
    return k.t()


def rhs_uniform_torch(n: int, nrhs: int = 1, seed: int = SEED_RHS, device: str = "cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    b = torch.empty((nrhs, n), dtype=torch.float64, device=device)
    b.uniform_(-1.0, 1.0, generator=g)
    return b.t() if nrhs > 1 else b[0]


def sha256(a: np.ndarray) -> str:
    """SHA-256 of the array's column-major bytes (records which bits a run used)."""
    return hashlib.sha256(np.asfortranarray(a).tobytes(order="F")).hexdigest()
