"""CPU oracle for the dense LU / Cholesky hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg import this package.  It shares no code with
the HIP library and never imports it.

Contents
  * ctypes bindings of ``liboracle.so`` (plain C, OpenMP, binary64):
    ``dgetrf``/``dgetrs`` (LU with partial pivoting, statements S1/S2 of
    Sec. 6.1), ``dpotrf``/``dpotrs`` (Cholesky listing, Sec. 6.2) and the
    reference encoders of the low-precision update formats.
  * the mixed-precision blocked factorizations, written step by step in
    numpy on top of those calls (not defined by the paper; see each docstring);
  * classical iterative refinement and the HPL scaled residual;
  * the I/O lower bounds of Sec. 6 (closed forms, one processor).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FMT_BF16, FMT_FP16, FMT_E4M3 = 1, 2, 3
FMT_NAMES = {"bf16": FMT_BF16, "fp16": FMT_FP16, "fp8e4m3": FMT_E4M3, "e4m3": FMT_E4M3}
EPS = 2.0 ** -53          # unit roundoff of binary64 (backward error, HPL residual)

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_fp = ctypes.POINTER(ctypes.c_float)


def lib():
    """Load liboracle.so (building it first if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(_LIB_PATH)
    L.oracle_set_threads.argtypes = [ctypes.c_int]
    L.oracle_get_threads.restype = ctypes.c_int
    L.oracle_host_triad_gbs.argtypes = [ctypes.c_long, ctypes.c_int]
    L.oracle_host_triad_gbs.restype = ctypes.c_double
    L.oracle_dgetrf.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _ip, ctypes.c_int]
    L.oracle_dgetrf.restype = ctypes.c_int
    L.oracle_dgetrs.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _ip, _dp, ctypes.c_int]
    L.oracle_dpotrf.argtypes = [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int]
    L.oracle_dpotrf.restype = ctypes.c_int
    L.oracle_dpotrs.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, ctypes.c_int]
    L.oracle_enc_bf16.argtypes = [ctypes.c_float]
    L.oracle_enc_bf16.restype = ctypes.c_uint16
    L.oracle_dec_bf16.argtypes = [ctypes.c_uint16]
    L.oracle_dec_bf16.restype = ctypes.c_double
    L.oracle_enc_f16.argtypes = [ctypes.c_double]
    L.oracle_enc_f16.restype = ctypes.c_uint16
    L.oracle_dec_f16.argtypes = [ctypes.c_uint16]
    L.oracle_dec_f16.restype = ctypes.c_double
    L.oracle_enc_e4m3.argtypes = [ctypes.c_double]
    L.oracle_enc_e4m3.restype = ctypes.c_uint8
    L.oracle_dec_e4m3.argtypes = [ctypes.c_uint8]
    L.oracle_dec_e4m3.restype = ctypes.c_double
    L.oracle_tile_scale_exp.argtypes = [ctypes.c_int, ctypes.c_float]
    L.oracle_tile_scale_exp.restype = ctypes.c_int
    L.oracle_quantize.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _fp, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, _ip]
    _lib = L
    return L


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def host_triad_gbs(n: int = 1 << 26, reps: int = 5) -> float:
    """Host memory bandwidth (GB/s) by a STREAM-style triad on all threads;
    reported beside the CPU baseline, not part of the method."""
    return float(lib().oracle_host_triad_gbs(int(n), int(reps)))


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), for the baseline report."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _f64(a: np.ndarray) -> np.ndarray:
    return np.array(a, dtype=np.float64, order="F", copy=True)


# --------------------------------------------------------------------------
# FP64 factorizations and solves (C)
# --------------------------------------------------------------------------

def dgetrf(a: np.ndarray, ksteps: int | None = None):
    """LU with partial pivoting of a copy of ``a`` (m x n).

    Returns (lu, ipiv, info): lu holds unit-lower L strictly below the
    diagonal and U on and above it, ipiv is 1-based (LAPACK interchanges),
    info = k+1 for the first exactly-zero pivot, else 0.  ``ksteps`` stops
    after that many elimination steps (trailing block = Schur complement).
    """
    lu = _f64(a)
    m, n = lu.shape
    kmax = min(m, n)
    ipiv = np.zeros(kmax, dtype=np.int32)
    ks = kmax if ksteps is None else int(ksteps)
    info = lib().oracle_dgetrf(m, n, lu.ctypes.data_as(_dp), max(1, m),
                               ipiv.ctypes.data_as(_ip), ks)
    return lu, ipiv, int(info)


def dgetrs(lu: np.ndarray, ipiv: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve A X = B from dgetrf's factors (B: n or n x nrhs)."""
    lu = np.asfortranarray(lu, dtype=np.float64)
    n = lu.shape[0]
    x = _f64(b.reshape(n, -1))
    ip = np.ascontiguousarray(ipiv, dtype=np.int32)
    lib().oracle_dgetrs(n, x.shape[1], lu.ctypes.data_as(_dp), max(1, n), ip.ctypes.data_as(_ip),
                        x.ctypes.data_as(_dp), max(1, n))
    return x.reshape(b.shape)


def dpotrf(a: np.ndarray, ksteps: int | None = None):
    """Lower Cholesky of a copy of ``a``; returns (l, info).

    Only the lower triangle is read or written: the strict upper triangle of
    the result is the input's, untouched.
    """
    l = _f64(a)
    n = l.shape[0]
    ks = n if ksteps is None else int(ksteps)
    info = lib().oracle_dpotrf(n, l.ctypes.data_as(_dp), max(1, n), ks)
    return l, int(info)


def dpotrs(l: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve A X = B from the lower Cholesky factor."""
    l = np.asfortranarray(l, dtype=np.float64)
    n = l.shape[0]
    x = _f64(b.reshape(n, -1))
    lib().oracle_dpotrs(n, x.shape[1], l.ctypes.data_as(_dp), max(1, n), x.ctypes.data_as(_dp), max(1, n))
    return x.reshape(b.shape)


# --------------------------------------------------------------------------
# Helpers on the factors
# --------------------------------------------------------------------------

def ipiv_to_perm(ipiv: np.ndarray, m: int) -> np.ndarray:
    """Row permutation p (0-based) such that (P A)[i] = A[p[i]]."""
    p = np.arange(m)
    for k, piv in enumerate(np.asarray(ipiv)):
        j = int(piv) - 1
        p[k], p[j] = p[j], p[k]
    return p


def split_lu(lu: np.ndarray):
    n = lu.shape[0]
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    return L, U


def lu_backward_error(a: np.ndarray, lu: np.ndarray, ipiv: np.ndarray) -> float:
    """||P A - L U||_F / (||A||_F * n * eps), eps = 2^-53."""
    n = a.shape[0]
    L, U = split_lu(np.asarray(lu, dtype=np.float64))
    p = ipiv_to_perm(ipiv, n)
    r = a[p, :] - L @ U
    return float(np.linalg.norm(r) / (np.linalg.norm(a) * n * EPS))


def chol_backward_error(a: np.ndarray, l: np.ndarray) -> float:
    """||A - L L^T||_F / (||A||_F * n * eps), both on the lower triangle's symmetric extension."""
    n = a.shape[0]
    L = np.tril(np.asarray(l, dtype=np.float64))
    As = np.tril(a) + np.tril(a, -1).T
    r = As - L @ L.T
    return float(np.linalg.norm(r) / (np.linalg.norm(As) * n * EPS))


def hpl_scaled_residual(a: np.ndarray, x: np.ndarray, b: np.ndarray) -> float:
    """max over columns of ||A x - b||_inf / (eps (||A||_inf ||x||_inf + ||b||_inf) n)."""
    n = a.shape[0]
    x2 = np.asarray(x, dtype=np.float64).reshape(n, -1)
    b2 = np.asarray(b, dtype=np.float64).reshape(n, -1)
    r = a @ x2 - b2
    anorm = np.abs(a).sum(axis=1).max()
    out = 0.0
    for c in range(x2.shape[1]):
        den = EPS * (anorm * np.abs(x2[:, c]).max() + np.abs(b2[:, c]).max()) * n
        out = max(out, float(np.abs(r[:, c]).max() / den))
    return out


def lu_flops(n: int) -> float:
    """Flop convention for LU throughput: 2 n^3 / 3."""
    return 2.0 * n ** 3 / 3.0


def chol_flops(n: int) -> float:
    """Flop convention for Cholesky throughput: n^3 / 3."""
    return n ** 3 / 3.0


def lu_step_flops(n: int, steps: int) -> float:
    """Exact flops of the first ``steps`` elimination steps of an n x n LU."""
    s = 0.0
    for k in range(min(n, steps)):
        r = n - k - 1
        s += r + 2.0 * r * r
    return s


def chol_step_flops(n: int, steps: int) -> float:
    """Exact flops of the first ``steps`` outer steps of an n x n Cholesky
    (square root, divisions, and the lower-triangle update)."""
    s = 0.0
    for k in range(min(n, steps)):
        r = n - k - 1
        s += 1 + r + r * (r + 1.0)
    return s


# --------------------------------------------------------------------------
# Quantizer reference (C)
# --------------------------------------------------------------------------

def enc_bf16(x: float) -> int:
    return int(lib().oracle_enc_bf16(float(x)))


def dec_bf16(c: int) -> float:
    return float(lib().oracle_dec_bf16(int(c)))


def enc_f16(x: float) -> int:
    return int(lib().oracle_enc_f16(float(x)))


def dec_f16(c: int) -> float:
    return float(lib().oracle_dec_f16(int(c)))


def enc_e4m3(x: float) -> int:
    return int(lib().oracle_enc_e4m3(float(x)))


def dec_e4m3(c: int) -> float:
    return float(lib().oracle_dec_e4m3(int(c)))


def tile_scale_exp(fmt: int, amax: float) -> int:
    return int(lib().oracle_tile_scale_exp(int(fmt), float(amax)))


def decode_table(fmt: int) -> np.ndarray:
    """Decoded values of every code of the format (float64)."""
    if fmt == FMT_E4M3:
        return np.array([dec_e4m3(c) for c in range(256)])
    dec = dec_bf16 if fmt == FMT_BF16 else dec_f16
    return np.array([dec(c) for c in range(65536)])


def quantize(fmt: int, x: np.ndarray, tm: int, tn: int):
    """Tile-quantize a float32 matrix; returns (codes, scale exponents).

    codes: uint16 (bf16/fp16) or uint8 (e4m3), same shape, column-major.
    exps : int32 array of shape (ceil(m/tm), ceil(n/tn)).
    """
    x = np.asfortranarray(x, dtype=np.float32)
    m, n = x.shape
    q = np.zeros((m, n), dtype=np.uint8 if fmt == FMT_E4M3 else np.uint16, order="F")
    mt, nt = -(-m // tm), -(-n // tn)
    e = np.zeros((mt, nt), dtype=np.int32, order="F")
    if m and n:
        lib().oracle_quantize(int(fmt), m, n, x.ctypes.data_as(_fp), max(1, m), int(tm), int(tn),
                              q.ctypes.data_as(ctypes.c_void_p), max(1, m), e.ctypes.data_as(_ip))
    return q, e


def dequantize(fmt: int, q: np.ndarray, e: np.ndarray, tm: int, tn: int) -> np.ndarray:
    """Exact float64 values dec(q) * 2^-e of a tile-quantized matrix."""
    table = decode_table(fmt)
    v = table[q.astype(np.int64)]
    m, n = q.shape
    ex = np.repeat(np.repeat(e, tm, axis=0), tn, axis=1)[:m, :n]
    return np.ldexp(v, -ex)


# --------------------------------------------------------------------------
# Mixed-precision blocked factorizations (numpy, step by step)
# --------------------------------------------------------------------------

# --------------------------------------------------------------------------
# Tournament pivoting (Sec. 7.3, "Tournament Pivoting" and "Pivoting in
# COnfLUX"; Table 1, row "pivoting")
# --------------------------------------------------------------------------

def gepp_rows(p: np.ndarray, rows: list, v: int) -> list:
    """The rows of ``p`` (indices) that LU with partial pivoting of the
    stacked rows ``p[rows]`` brings to the top, in pivot order (at most v).
    The local decomposition each participant of a tournament round runs."""
    rows = list(rows)
    k = min(v, len(rows), p.shape[1])
    _, ipiv, _ = dgetrf(p[rows, :], ksteps=k)
    order = list(rows)
    for i in range(k):
        q = int(ipiv[i]) - 1
        order[i], order[q] = order[q], order[i]
    return order[:k]


def tournament_pivots(p: np.ndarray, v: int, block: int, fanin: int) -> list:
    """The v pivot rows of the block column ``p`` (m x v, original values)
    chosen by tournament pivoting: every group of ``block`` consecutive rows
    picks v candidates by a local LU with partial pivoting; then, round by
    round, the candidate sets are taken ``fanin`` at a time (in order,
    stacked in order) and a local LU of their original rows keeps v of them,
    until one set is left.  Returns row indices in pivot order."""
    m = p.shape[0]
    sets = [gepp_rows(p, range(s, min(m, s + block)), v) for s in range(0, m, block)]
    while len(sets) > 1:
        sets = [gepp_rows(p, [r for st in sets[i:i + fanin] for r in st], v)
                for i in range(0, len(sets), fanin)]
    return sets[0]


def calu_panel(a: np.ndarray, leaf: int = 32, block: int = 256, fanin: int = 8):
    """LU of an m x n block column (m >= n) whose pivots are chosen by
    tournament pivoting on each ``leaf``-wide column block in turn.

    For each leaf at column c0 (width w): the tournament over the current
    rows [c0, m) of the leaf's columns names the w pivot rows; they are
    interchanged into rows c0.. c0+w-1 in pivot order (LAPACK-style swap
    sequence, applied to all columns); the leaf's columns are then
    eliminated without further interchanges (a zero pivot is recorded in
    info and its column left unscaled); U12 = L11^-1 A12 and A22 -= L21 U12
    update the columns right of the leaf.  With block >= m every tournament
    is a single local LU, so the result is LU with partial pivoting.
    Returns (lu, ipiv 1-based, info)."""
    from scipy.linalg import solve_triangular  # library primitive: triangular solve

    lu = _f64(a)
    m, n = lu.shape
    kmax = min(m, n)
    ipiv = np.zeros(kmax, dtype=np.int32)
    info = 0
    for c0 in range(0, kmax, leaf):
        w = min(leaf, kmax - c0)
        order = tournament_pivots(lu[c0:, c0:c0 + w], w, block, fanin)
        at = list(range(m - c0))       # at[i]: original (leaf-relative) row now at position i
        where = {r: r for r in at}     # where[r]: position of original row r
        for j, r in enumerate(order):
            q = where[r]
            ipiv[c0 + j] = c0 + q + 1
            if q != j:
                lu[[c0 + j, c0 + q], :] = lu[[c0 + q, c0 + j], :]
                rj = at[j]
                at[j], at[q] = r, rj
                where[r], where[rj] = j, q
        for k in range(c0, c0 + w):
            piv = lu[k, k]
            if piv == 0.0:
                if not info:
                    info = k + 1
                continue
            lu[k + 1:, k] /= piv
            lu[k + 1:, k + 1:c0 + w] -= np.outer(lu[k + 1:, k], lu[k, k + 1:c0 + w])
        if c0 + w < n:
            l11 = np.tril(lu[c0:c0 + w, c0:c0 + w], -1) + np.eye(w)
            lu[c0:c0 + w, c0 + w:] = solve_triangular(l11, lu[c0:c0 + w, c0 + w:], lower=True, unit_diagonal=True)
            lu[c0 + w:, c0 + w:] -= lu[c0 + w:, c0:c0 + w] @ lu[c0:c0 + w, c0 + w:]
    return lu, ipiv, info


def _laswp_rows(w: np.ndarray, cols: slice, k0: int, piv: np.ndarray) -> None:
    """Apply interchanges (0-based rows k0+i <-> piv[i]) in order to w[:, cols]."""
    for i, p in enumerate(piv):
        r = k0 + i
        if p != r:
            tmp = w[r, cols].copy()
            w[r, cols] = w[p, cols]
            w[p, cols] = tmp


def mixed_getrf(a: np.ndarray, nb: int, fmt: int, tm: int, tn: int, tournament=None):
    """Blocked right-looking LU with a low-precision trailing update.

    Not defined by the paper (it only cites low-precision LU with refinement
    as related work); the steps follow the blocked right-looking schedule
    whose dominant step is the Schur-complement update (Sec. 7):
      W = binary32(A)
      for each panel of width nb at column k:
        P = binary64(W[k:, k:k+nb]); LU with partial pivoting of P (dgetrf);
        W[k:, panel] = binary32(P); interchanges applied to W's other columns
        U12 = L11^-1 binary64(W[k:k+nb, k+nb:])  (binary64), W12 = binary32(U12)
        L21, U12 (binary32) tile-quantized: L21 in tm x nb tiles, U12 in nb x tn
        W22 = binary32(binary64(W22) - dq(L21) @ dq(U12))
    With ``tournament = (leaf, block, fanin)`` the panel's pivots are chosen
    by tournament pivoting (calu_panel) instead of partial pivoting.
    Returns (w float32, ipiv 1-based, info).
    """
    from scipy.linalg import solve_triangular  # library primitive: triangular solve

    n = a.shape[0]
    w = np.asfortranarray(a, dtype=np.float32).copy(order="F")
    ipiv = np.zeros(n, dtype=np.int32)
    info = 0
    for k in range(0, n, nb):
        kb = min(nb, n - k)
        p = w[k:, k:k + kb].astype(np.float64)
        pl, pp, pinfo = dgetrf(p) if tournament is None else calu_panel(p, *tournament)
        if pinfo and not info:
            info = k + pinfo
        w[k:, k:k + kb] = pl.astype(np.float32)
        ipiv[k:k + kb] = pp + k
        piv0 = (pp - 1) + k
        _laswp_rows(w, slice(0, k), k, piv0)
        _laswp_rows(w, slice(k + kb, n), k, piv0)
        if k + kb < n:
            l11 = np.tril(pl[:kb, :kb], -1) + np.eye(kb)
            u12 = solve_triangular(l11, w[k:k + kb, k + kb:].astype(np.float64), lower=True,
                                   unit_diagonal=True)
            w[k:k + kb, k + kb:] = u12.astype(np.float32)
            l21 = w[k + kb:, k:k + kb]
            u12f = w[k:k + kb, k + kb:]
            qa, ea = quantize(fmt, l21, tm, kb)
            qb, eb = quantize(fmt, u12f, kb, tn)
            prod = dequantize(fmt, qa, ea, tm, kb) @ dequantize(fmt, qb, eb, kb, tn)
            w[k + kb:, k + kb:] = (w[k + kb:, k + kb:].astype(np.float64) - prod).astype(np.float32)
    return w, ipiv, info


def mixed_potrf(a: np.ndarray, nb: int, fmt: int, tm: int):
    """Blocked right-looking lower Cholesky with a low-precision SYRK update.

      W = binary32(lower(A))
      for each diagonal block of width nb at k:
        L11 = chol(binary64(W11)) (dpotrf); W11 = binary32(L11)
        L21 = binary64(W21) L11^-T (binary64); W21 = binary32(L21)
        L21 tile-quantized in tm x nb tiles (the transposed operand reuses the
        same tiles, so each product carries the two tiles' scales)
        lower(W22) = binary32(binary64(W22) - dq(L21) @ dq(L21)^T)
    Returns (w float32 with the factor in its lower triangle, info).
    """
    from scipy.linalg import solve_triangular

    n = a.shape[0]
    w = np.asfortranarray(np.tril(a), dtype=np.float32).copy(order="F")
    for k in range(0, n, nb):
        kb = min(nb, n - k)
        d = w[k:k + kb, k:k + kb].astype(np.float64)
        l11, dinfo = dpotrf(d)
        if dinfo:
            return w, k + dinfo
        l11 = np.tril(l11)
        w[k:k + kb, k:k + kb] = l11.astype(np.float32)
        if k + kb < n:
            a21 = w[k + kb:, k:k + kb].astype(np.float64)
            l21 = solve_triangular(l11, a21.T, lower=True).T
            w[k + kb:, k:k + kb] = l21.astype(np.float32)
            qa, ea = quantize(fmt, w[k + kb:, k:k + kb], tm, kb)
            dl = dequantize(fmt, qa, ea, tm, kb)
            upd = w[k + kb:, k + kb:].astype(np.float64) - dl @ dl.T
            w[k + kb:, k + kb:] = np.tril(upd).astype(np.float32)
    return w, 0


def solve_with_lu32(w: np.ndarray, ipiv: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve with binary32 LU factors, arithmetic in binary64."""
    return dgetrs(w.astype(np.float64), ipiv, b)


def solve_with_chol32(w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve with a binary32 lower Cholesky factor, arithmetic in binary64."""
    return dpotrs(np.tril(w).astype(np.float64), b)


def iterative_refinement(a: np.ndarray, b: np.ndarray, solve, max_iter: int = 30,
                         target: float = 16.0):
    """Classical iterative refinement to an HPL scaled residual <= target.

    x0 = solve(b); then repeat: r = b - A x (binary64, original A); stop if
    the scaled residual is <= target; else x += solve(r).  Stops without
    convergence after max_iter corrections or when the residual has not
    halved over three corrections.  Returns (x, corrections, residual, ok).
    """
    x = solve(b)
    hist = []
    for it in range(max_iter + 1):
        res = hpl_scaled_residual(a, x, b)
        hist.append(res)
        if res <= target:
            return x, it, res, True
        if it == max_iter or (len(hist) > 3 and hist[-1] > 0.5 * hist[-4]):
            return x, it, res, False
        r = b - a @ x
        x = x + solve(r)
    return x, max_iter, hist[-1], False


# --------------------------------------------------------------------------
# Preconditioned conjugate gradients with a low-precision Cholesky factor
# (the fallback when classical refinement fails on an SPD system)
# --------------------------------------------------------------------------

def shift_diagonal(a: np.ndarray, sigma: float) -> np.ndarray:
    """A + sigma * diag(A) in binary64 (each a_ii * (1 + sigma), one rounding;
    sigma a power of two, so 1 + sigma is exact)."""
    out = np.array(a, dtype=np.float64, order="F", copy=True)
    d = np.diag(out) * (1.0 + sigma)
    out[np.diag_indices(out.shape[0])] = d
    return out


def pcg(a: np.ndarray, b: np.ndarray, precond, max_iter: int = 400, target: float = 16.0,
        x0: np.ndarray | None = None, history: bool = False):
    """Preconditioned conjugate gradients for the SPD system A X = B, every
    column on its own, binary64 (the method of Hestenes and Stiefel with a
    preconditioner M^-1 applied by ``precond``).

      x = x0 (default M^-1 b); r = b - A x; z = M^-1 r; p = z; rho = r.z
      repeat: q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q
              stop if the HPL scaled residual of b - A x is <= target
              z = M^-1 r; rho' = r.z; beta = rho' / rho; p = z + beta p
    A column whose p.q (or rho) is zero takes alpha (or beta) = 0: it has
    converged exactly.  Returns (x, iterations, residual, converged[, the
    iterates x_1, x_2, ... when history])."""
    a = np.asarray(a, dtype=np.float64)
    b2 = np.asarray(b, dtype=np.float64).reshape(a.shape[0], -1)
    x = precond(b2.copy()) if x0 is None else np.array(x0, dtype=np.float64).reshape(b2.shape)
    r = b2 - a @ x
    hist = []
    res = hpl_scaled_residual(a, x, b2)
    if res <= target:
        return (x.reshape(b.shape), 0, res, True) + ((hist,) if history else ())
    z = precond(r.copy())
    p = z.copy()
    rho = np.sum(r * z, axis=0)
    for it in range(1, max_iter + 1):
        q = a @ p
        pq = np.sum(p * q, axis=0)
        alpha = np.divide(rho, pq, out=np.zeros_like(rho), where=pq != 0)
        x = x + alpha * p
        r = r - alpha * q
        if history:
            hist.append(x.reshape(b.shape).copy())
        res = hpl_scaled_residual(a, x, b2)
        if res <= target:
            return (x.reshape(b.shape), it, res, True) + ((hist,) if history else ())
        z = precond(r.copy())
        rho_new = np.sum(r * z, axis=0)
        beta = np.divide(rho_new, rho, out=np.zeros_like(rho), where=rho != 0)
        rho = rho_new
        p = z + beta * p
    return (x.reshape(b.shape), max_iter, res, False) + ((hist,) if history else ())


def shift_schedule(fmt: int, attempts: int = 6):
    """Diagonal shifts tried after a low-precision Cholesky breaks down:
    sigma_j = u * 4^j (j = 0, 1, ...), u the format's unit roundoff (the shift
    of a low-precision Cholesky preconditioner scales with u)."""
    u = {FMT_BF16: 2.0 ** -8, FMT_FP16: 2.0 ** -11, FMT_E4M3: 2.0 ** -4}[fmt]
    return [u * 4.0 ** j for j in range(attempts)]


def spd_solve_shifted_pcg(a: np.ndarray, b: np.ndarray, nb: int, fmt: int, tm: int, max_iter: int = 400,
                          target: float = 16.0):
    """The fallback for an SPD system when classical refinement with the
    low-precision Cholesky fails: factor A + sigma diag(A) with the
    low-precision update (mixed_potrf) for sigma = 0, then the shifts of
    shift_schedule until one factorization completes, and solve A X = B by
    pcg() with that factor as the preconditioner.  Returns (x, sigma,
    factorizations, iterations, residual, converged)."""
    for f, sigma in enumerate([0.0] + shift_schedule(fmt)):
        w, info = mixed_potrf(shift_diagonal(a, sigma) if sigma else a, nb, fmt, tm)
        if info == 0:
            x, it, res, ok = pcg(a, b, lambda r: solve_with_chol32(w, r), max_iter, target)
            return x, sigma, f + 1, it, res, ok
    return None, None, f + 1, 0, float("inf"), False


# --------------------------------------------------------------------------
# I/O lower bounds (Sec. 6, one processor, in elements)
# --------------------------------------------------------------------------

def io_lower_bound_elems(kind: int, n: float, m: float) -> float:
    """Sequential (P = 1) I/O lower bound in elements for fast memory M.

    kind 0 (LU, Sec. 6.1): (2N^3 - 6N^2 + 4N) / (3 sqrt(M)) + N(N-1)/2.
    kind 1 (Cholesky, Sec. 6.2): N^3 / (3 sqrt(M)) + N^2 / 2 + N.
    """
    sm = math.sqrt(m)
    if kind == 0:
        return (2 * n ** 3 - 6 * n ** 2 + 4 * n) / (3 * sm) + n * (n - 1) / 2
    return n ** 3 / (3 * sm) + n ** 2 / 2 + n


def chi_closed_form(x: float) -> float:
    """Largest S2 subcomputation |H| = (X/3)^(3/2) for dominator size X (Sec. 6.1)."""
    return (x / 3.0) ** 1.5


# --------------------------------------------------------------------------
# General I/O lower bound of a DAAP statement or program (Sec. 3 and 4)
# --------------------------------------------------------------------------

def daap_chi(nvars: int, accesses, weights, x: float):
    """chi(X) of Sec. 3.2: the largest subcomputation prod_t |D^t| whose
    dominator set sum_j w_j prod_{t in access j} |D^t| fits in X, every
    |D^t| >= 1 (continuous relaxation).  ``accesses`` lists, per input
    access, the indices of its distinct iteration variables; ``weights``
    the factor of each access (1, or 1/rho_S for the output of a producer
    S, Corollary of Sec. 4.2).  Solved in logarithms y_t = ln |D^t| (a convex
    program) with scipy's SLSQP.  Returns (chi, [|D^t|])."""
    from scipy.optimize import minimize

    a = np.zeros((len(accesses), nvars))
    for j, vs in enumerate(accesses):
        for t in vs:
            a[j, t] = 1.0
    w = np.asarray(weights, dtype=np.float64)
    lx = math.log(x)

    def h(y):
        return float(np.log(np.sum(w * np.exp(a @ y))))

    def hgrad(y):
        e = w * np.exp(a @ y)
        return (e / e.sum()) @ a

    y0 = np.zeros(nvars)
    res = minimize(lambda y: -float(np.sum(y)), y0, jac=lambda y: -np.ones(nvars), method="SLSQP",
                   bounds=[(0.0, None)] * nvars,
                   constraints=[{"type": "ineq", "fun": lambda y: lx - h(y), "jac": lambda y: -hgrad(y)}],
                   options={"ftol": 1e-14, "maxiter": 500})
    y = np.maximum(res.x, 0.0)
    return float(math.exp(np.sum(y))), [float(math.exp(v)) for v in y]


def daap_statement_bound(nvars: int, accesses, weights, nvertices: float, m: float, u: int = 0) -> dict:
    """I/O lower bound of one statement (Sec. 3.2): rho = min over X > M of
    chi(X) / (X - M) (Lemma of Sec. 3, X_0 its argmin), capped at 1/u when
    every compute vertex has u out-degree-one input predecessors (Lemma of
    Sec. 3.2); Q >= |V| / rho.  The search runs over ln X (bounded scalar
    minimization) between the smallest feasible X and 2^40 M."""
    from scipy.optimize import minimize_scalar

    lo = max(m, float(np.sum(weights))) * (1 + 1e-9)
    hi = m * 2.0 ** 40

    def rho_of(lx):
        x = math.exp(lx)
        return daap_chi(nvars, accesses, weights, x)[0] / (x - m)

    r = minimize_scalar(rho_of, bounds=(math.log(lo), math.log(hi)), method="bounded",
                        options={"xatol": 1e-10})
    x0 = math.exp(r.x)
    chi, tiles = daap_chi(nvars, accesses, weights, x0)
    rho = chi / (x0 - m)
    if u > 0:
        rho = min(rho, 1.0 / u)
    sizes = [w * math.prod(tiles[t] for t in vs) for vs, w in zip(accesses, weights)]
    return {"rho": rho, "x0": x0, "chi": chi, "tiles": tiles, "access_sizes": sizes, "q": nvertices / rho}


def daap_program_bound(statements, m: float) -> float:
    """I/O lower bound of a program of several statements (Sec. 4): the sum
    of the statements' bounds minus, for every input array shared by several
    statements (Case I), the loads that can be shared: each statement alone
    loads |A(R_max(X_0))| |V| / |V_max| elements of the array in its optimal
    schedule, and at least the largest of these loads remain, so the sum
    minus that maximum is subtracted (for two statements: the minimum).
    Output reuse (Case II) enters through the access weights.  Each statement
    is a dict with keys nvars, accesses, weights, nvertices, u and arrays
    (the array id of each access)."""
    total = 0.0
    loads = {}
    for s in statements:
        r = daap_statement_bound(s["nvars"], s["accesses"], s["weights"], s["nvertices"], m, s.get("u", 0))
        total += r["q"]
        nsub = s["nvertices"] / r["chi"]
        for arr, size in zip(s["arrays"], r["access_sizes"]):
            loads.setdefault(arr, []).append(size * nsub)
    for arr, ls in loads.items():
        if len(ls) > 1:
            total -= sum(ls) - max(ls)
    return total
