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


# ----------------------------------------------------------------- large n
# Checks of GPU results at sizes where the CPU oracle cannot factor the whole
# matrix: invariants evaluated with torch's FP64 matrix products (rocBLAS),
# which share nothing with the library's kernels.

def perm_from_ipiv(ipiv, n):
    """Row permutation p (0-based): (P A)[i] = A[p[i]] for LAPACK interchanges."""
    p = np.arange(n)
    for k, piv in enumerate(np.asarray(ipiv)):
        j = int(piv) - 1
        p[k], p[j] = p[j], p[k]
    return p


def lu_backward_error_torch(torch, A0, LU, ipiv, bs=8192):
    """||P A - L U||_F / (||A||_F n eps) in FP64 on the GPU, in bs x bs blocks
    (masks by broadcasting; no single kernel touches more than one block).

    A0, LU: n x n device tensors (any strides), ipiv: host int array."""
    n = A0.shape[0]
    dev = A0.device
    perm = torch.from_numpy(perm_from_ipiv(ipiv, n)).to(dev)
    ss = torch.zeros((), dtype=torch.float64, device=dev)
    an = torch.zeros((), dtype=torch.float64, device=dev)
    zero = torch.zeros((), dtype=torch.float64, device=dev)
    one = torch.ones((), dtype=torch.float64, device=dev)
    for c0 in range(0, n, bs):
        c1 = min(n, c0 + bs)
        # U[:c1, c0:c1]: entries with row <= col
        Uj = torch.where(torch.arange(0, c1, device=dev)[:, None] <= torch.arange(c0, c1, device=dev)[None, :],
                         LU[:c1, c0:c1], zero).contiguous()
        for r0 in range(0, n, bs):
            r1 = min(n, r0 + bs)
            kk = min(r1, c1)  # L[i, p] = 0 for p > i, U[p, j] = 0 for p > j
            rr = torch.arange(r0, r1, device=dev)[:, None]
            pp = torch.arange(0, kk, device=dev)[None, :]
            Ls = torch.where(pp < rr, LU[r0:r1, :kk], torch.where(pp == rr, one, zero)).contiguous()
            Ab = A0[:, c0:c1][perm[r0:r1]]
            R = Ab - Ls @ Uj[:kk]
            ss += (R * R).sum()
            an += (Ab * Ab).sum()
            del Ls, Ab, R
        del Uj
    return float(torch.sqrt(ss) / (torch.sqrt(an) * n * EPS))


def chol_backward_error_torch(torch, A0, L, bs=8192):
    """||A - L L^T||_F / (||A||_F n eps) on the lower triangle's symmetric
    extension (as the oracle defines it), FP64 on the GPU, in bs x bs blocks
    of the lower triangle (off-diagonal entries weighted twice)."""
    n = A0.shape[0]
    dev = A0.device
    ss = torch.zeros((), dtype=torch.float64, device=dev)
    an = torch.zeros((), dtype=torch.float64, device=dev)
    zero = torch.zeros((), dtype=torch.float64, device=dev)
    for c0 in range(0, n, bs):
        c1 = min(n, c0 + bs)
        cj = torch.arange(c0, c1, device=dev)[:, None]
        pj = torch.arange(0, c1, device=dev)[None, :]
        Lj = torch.where(pj <= cj, L[c0:c1, :c1], zero).contiguous()  # rows c0:c1 of lower L
        for r0 in range(c0, n, bs):
            r1 = min(n, r0 + bs)
            ri = torch.arange(r0, r1, device=dev)[:, None]
            Li = torch.where(pj <= ri, L[r0:r1, :c1], zero).contiguous()
            cc = torch.arange(c0, c1, device=dev)[None, :]
            low = cc <= ri
            w = torch.where(cc == ri, 1.0, 2.0).to(torch.float64) * low
            Ab = torch.where(low, A0[r0:r1, c0:c1], zero)
            R = Ab - Li @ Lj.t()
            ss += (w * R * R).sum()
            an += (w * Ab * Ab).sum()
            del Li, Ab, R, w
        del Lj
    return float(torch.sqrt(ss) / (torch.sqrt(an) * n * EPS))


def lu_partial_tolerance(lu_k, k, n_full):
    """Elementwise tolerance for the first k steps of an n_full x n_full LU,
    from the oracle's k-step result on a column subset (first k columns then
    sampled ones): 16 n eps (|L||U|)_ij, divided by |u_jj| for L entries.
    Entries outside L[:, :k] and U[:k, :] get an infinite tolerance."""
    m, c = lu_k.shape
    L = np.tril(lu_k[:, :k], -1)
    L[np.arange(k), np.arange(k)] = 1.0
    U = np.triu(lu_k[:k, :])
    tol = np.full((m, c), np.inf)
    LU = np.abs(L) @ np.abs(U)
    t = 16 * n_full * EPS * LU + 1e-300
    d = np.abs(np.diag(U[:, :k]))
    d[d == 0] = 1.0
    low = np.tril(np.ones((m, k), dtype=bool), -1)
    tl = t[:, :k] / d[None, :]
    tol[:, :k] = np.where(low, tl, np.inf)
    upper = np.triu(np.ones((k, c), dtype=bool))
    tol[:k, :] = np.where(upper, t[:k, :], tol[:k, :])
    return tol
