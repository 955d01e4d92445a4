"""Python binding of libcdnafact: dense LU / Cholesky factorizations and
solves, mixed-precision solvers and batched small factorizations for AMD
MI355X (gfx950).

Argument marshalling only: every step runs in the HIP kernels of
``libcdnafact.so`` (built in-tree by ``build.py``).  torch supplies device
memory and the current stream.  Matrices are column-major: a 2-D tensor must
have stride(0) == 1 (e.g. from :func:`cm_empty` / :func:`to_device`); its
leading dimension is stride(1).  1-D tensors are single columns.

The library is loaded after ``import torch`` so that both share one HIP
runtime.  If ``libcdnafact.so`` is missing this module raises: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcdnafact.so")

CDF_OK, CDF_ERR_INVALID_ARG, CDF_ERR_HIP, CDF_ERR_ALLOC, CDF_ERR_NOT_CONVERGED, CDF_ERR_UNSUPPORTED, \
    CDF_ERR_TIMEOUT = range(7)
CDF_INFO_TIMEOUT = -1000  # device info of an LU whose panel exchange ran out of its wait budget
UPD = {"fp64": 0, "bf16": 1, "fp16": 2, "fp8e4m3": 3, "e4m3": 3}
PARAM = {"lu_nb": 0, "chol_nb": 1, "lu_leaf_rows": 2, "mixed_nb": 3, "vbatch_nb": 4, "vbatch_wg_per_cu": 5,
         "gemm_wg_per_cu": 6, "lu_u12": 7, "leaf_wait_us": 8, "test_exchange_fail": 9, "spd_refine": 10,
         "pcg_max_iter": 11, "gemm_tile": 12, "lu_pivot": 13, "tourn_block": 14, "tourn_fanin": 15}
REFINE = {0: None, 1: "classical", 2: "pcg"}
F64, F32 = 0, 1

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_double_p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i = ctypes.c_int
_lib = None


class CdfError(RuntimeError):
    def __init__(self, name, status, bad_arg=0):
        self.status = status
        self.bad_arg = bad_arg
        msg = f"{name} failed: {_lib.cdf_status_string(status).decode()}"
        if bad_arg:
            msg += f" (argument {bad_arg})"
        super().__init__(msg)


DAAP_MAX = 8  # CDF_DAAP_MAX_VARS, CDF_DAAP_MAX_ACCESSES


class DaapStatement(ctypes.Structure):
    _fields_ = [("nvars", ctypes.c_int), ("naccesses", ctypes.c_int),
                ("access_vars", ctypes.c_uint * DAAP_MAX), ("access_weight", ctypes.c_double * DAAP_MAX),
                ("array_id", ctypes.c_int * DAAP_MAX), ("u", ctypes.c_int), ("nvertices", ctypes.c_double)]


class DaapResult(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("x0", ctypes.c_double), ("chi", ctypes.c_double), ("q", ctypes.c_double),
                ("tile", ctypes.c_double * DAAP_MAX), ("access", ctypes.c_double * DAAP_MAX)]


def lib() -> ctypes.CDLL:
    """Load libcdnafact.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: run paper_2108_09337_amd/build.py (or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "cdf_create": (_i, [ctypes.POINTER(_vp)]),
        "cdf_destroy": (_i, [_vp]),
        "cdf_set_stream": (_i, [_vp, _vp]),
        "cdf_set_workspace_limit": (_i, [_vp, ctypes.c_size_t]),
        "cdf_workspace_bytes": (ctypes.c_size_t, [_vp]),
        "cdf_last_bad_arg": (_i, [_vp]),
        "cdf_status_string": (ctypes.c_char_p, [_i]),
        "cdf_device_status": (_i, [_vp]),
        "cdf_mixed_report": (_i, [_vp, _c_int_p, _c_double_p, _c_int_p, _c_int_p, _c_int_p]),
        "cdf_set_param": (_i, [_vp, _i, _i]),
        "cdf_get_param": (_i, [_vp, _i]),
        "cdf_dgetrf": (_i, [_vp, _i, _vp, _i, _vp, _vp]),
        "cdf_dgetrf_noalloc": (_i, [_vp, _i, _vp, _i, _vp, _vp]),
        "cdf_dgetrs": (_i, [_vp, ctypes.c_char, _i, _i, _vp, _i, _vp, _vp, _i]),
        "cdf_dpotrf": (_i, [_vp, ctypes.c_char, _i, _vp, _i, _vp]),
        "cdf_dpotrs": (_i, [_vp, ctypes.c_char, _i, _i, _vp, _i, _vp, _i]),
        "cdf_dgesv_mixed": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i, _i, _c_int_p, _c_double_p, _vp]),
        "cdf_dposv_mixed": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i, _i, _c_int_p, _c_double_p, _vp]),
        "cdf_sgetrf_mixed": (_i, [_vp, _i, _i, _vp, _i, _vp, _i, _vp, _vp]),
        "cdf_spotrf_mixed": (_i, [_vp, _i, ctypes.c_char, _i, _vp, _i, _vp, _i, _vp]),
        "cdf_quantize": (_i, [_vp, _i, _i, _i, _vp, _i, _i, _i, _vp, _i, _vp]),
        "cdf_lowp_update": (_i, [_vp, _i, _i, _i, _i, _vp, _i, _vp, _vp, _i, _vp, _vp, _i]),
        "cdf_update_tile": (_i, [_i]),
        "cdf_dgemm_update": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i]),
        "cdf_vbatch_plan_create": (_i, [_vp, _i, _c_int_p, _c_int_p, _i, ctypes.POINTER(_vp)]),
        "cdf_vbatch_run": (_i, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "cdf_vbatch_plan_destroy": (_i, [_vp]),
        "cdf_io_lower_bound_elems": (ctypes.c_double, [_i, ctypes.c_double, ctypes.c_double]),
        "cdf_daap_chi": (_i, [ctypes.POINTER(DaapStatement), ctypes.c_double, _c_double_p, _c_double_p]),
        "cdf_daap_statement_bound": (_i, [ctypes.POINTER(DaapStatement), ctypes.c_double,
                                          ctypes.POINTER(DaapResult)]),
        "cdf_daap_program_bound": (_i, [_i, ctypes.POINTER(DaapStatement), ctypes.c_double, _c_double_p]),
        "cdf_profile_begin": (_i, [_vp]),
        "cdf_profile_end": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_longlong), _c_double_p, _c_double_p, _c_double_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


# ---------------------------------------------------------------- handles

class Handle:
    """A library handle bound to one device; calls run on torch's current stream."""

    def __init__(self, device=None):
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
        self.device = dev
        with torch.cuda.device(dev):
            h = _vp()
            st = lib().cdf_create(ctypes.byref(h))
            if st != CDF_OK:
                raise CdfError("cdf_create", st)
        self._h = h

    @property
    def ptr(self):
        return self._h

    def bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        lib().cdf_set_stream(self._h, _vp(s))
        return self._h

    def set_param(self, name: str, value: int):
        _check("cdf_set_param", lib().cdf_set_param(self._h, PARAM[name], int(value)), self._h)

    def get_param(self, name: str) -> int:
        return int(lib().cdf_get_param(self._h, PARAM[name]))

    def set_workspace_limit(self, nbytes: int):
        lib().cdf_set_workspace_limit(self._h, int(nbytes))

    def workspace_bytes(self) -> int:
        return int(lib().cdf_workspace_bytes(self._h))

    def close(self):
        if self._h:
            lib().cdf_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict = {}


def handle(device=None) -> Handle:
    """The handle for (device, torch's current stream on it).

    One handle per stream keeps calls that may overlap in time (different
    streams) on separate workspaces and grid-barrier counters.
    """
    idx = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    key = (idx, torch.cuda.current_stream(idx).cuda_stream)
    h = _handles.get(key)
    if h is None:
        h = _handles[key] = Handle(idx)
    return h


def _check(name, status, h):
    if status != CDF_OK:
        raise CdfError(name, status, lib().cdf_last_bad_arg(h) if h else 0)


def _ld(t: torch.Tensor) -> int:
    if t.dim() == 1:
        return max(1, t.shape[0])
    if t.shape[1] > 1 and t.stride(0) != 1:
        raise ValueError("matrix tensors must be column-major (stride(0) == 1)")
    return max(1, t.stride(1) if t.shape[1] > 1 else t.shape[0])


def _cols(t: torch.Tensor) -> int:
    return 1 if t.dim() == 1 else t.shape[1]


def _p(t):
    return None if t is None else _vp(t.data_ptr())


# ---------------------------------------------------------------- helpers

def cm_empty(rows: int, cols: int, dtype=torch.float64, device="cuda") -> torch.Tensor:
    """Uninitialised column-major (rows x cols) tensor."""
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def to_device(a: np.ndarray, dtype=torch.float64, device="cuda") -> torch.Tensor:
    """Copy a numpy matrix (or vector) to a column-major device tensor."""
    if a.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)
    t = cm_empty(a.shape[0], a.shape[1], dtype, device)
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)).to(dtype))
    return t


def to_host(t: torch.Tensor) -> np.ndarray:
    """Device tensor -> numpy (column-major for matrices)."""
    a = t.detach().cpu()
    return np.asfortranarray(a.numpy()) if a.dim() == 2 else a.numpy().copy()


# ---------------------------------------------------------------- FP64 path

def dgetrf(A: torch.Tensor, ipiv: torch.Tensor, info: torch.Tensor, h: Handle | None = None) -> None:
    """In-place LU with partial pivoting (see cdf_dgetrf)."""
    h = h or handle(A.device)
    n = A.shape[0]
    _check("cdf_dgetrf", lib().cdf_dgetrf(h.bind_stream(), n, _p(A), _ld(A), _p(ipiv), _p(info)), h.ptr)


def dgetrf_noalloc(A: torch.Tensor, ipiv: torch.Tensor, info: torch.Tensor, h: Handle | None = None) -> None:
    """In-place LU that allocates nothing (see cdf_dgetrf_noalloc)."""
    h = h or handle(A.device)
    n = A.shape[0]
    _check("cdf_dgetrf_noalloc", lib().cdf_dgetrf_noalloc(h.bind_stream(), n, _p(A), _ld(A), _p(ipiv), _p(info)),
           h.ptr)


def dgetrs(A: torch.Tensor, ipiv: torch.Tensor, B: torch.Tensor, trans: str = "N", h: Handle | None = None) -> None:
    h = h or handle(A.device)
    n = A.shape[0]
    _check("cdf_dgetrs", lib().cdf_dgetrs(h.bind_stream(), trans.encode(), n, _cols(B), _p(A), _ld(A), _p(ipiv),
                                          _p(B), _ld(B)), h.ptr)


def dpotrf(A: torch.Tensor, info: torch.Tensor, uplo: str = "L", h: Handle | None = None) -> None:
    h = h or handle(A.device)
    n = A.shape[0]
    _check("cdf_dpotrf", lib().cdf_dpotrf(h.bind_stream(), uplo.encode(), n, _p(A), _ld(A), _p(info)), h.ptr)


def dpotrs(A: torch.Tensor, B: torch.Tensor, uplo: str = "L", h: Handle | None = None) -> None:
    h = h or handle(A.device)
    n = A.shape[0]
    _check("cdf_dpotrs", lib().cdf_dpotrs(h.bind_stream(), uplo.encode(), n, _cols(B), _p(A), _ld(A), _p(B),
                                          _ld(B)), h.ptr)


def dgemm_update(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, h: Handle | None = None) -> None:
    """C <- C - A B (FP64, matrix cores)."""
    h = h or handle(C.device)
    m, k = A.shape[0], _cols(A)
    n = _cols(C)
    _check("cdf_dgemm_update", lib().cdf_dgemm_update(h.bind_stream(), m, n, k, _p(A), _ld(A), _p(B), _ld(B),
                                                      _p(C), _ld(C)), h.ptr)


GEMM_KERNELS = {"nn": 0, "nt": 1, "tn": 2, "tt": 3, "syrk": 4, "u12": 5}


def device_status(h: Handle | None = None) -> int:
    """Synchronize the handle's streams; CDF_ERR_TIMEOUT if the last LU's panel
    exchange ran out of its wait budget, else CDF_OK (see cdf_device_status)."""
    h = h or handle()
    return int(lib().cdf_device_status(h.ptr))


def profile_begin(h: Handle | None = None) -> None:
    """Start timing every FP64 update-GEMM launch of this handle's calls (HIP events on its stream)."""
    h = h or handle()
    _check("cdf_profile_begin", lib().cdf_profile_begin(h.ptr), h.ptr)


def profile_end(kernel: str = "nn", h: Handle | None = None) -> dict:
    """Stop timing; launches, summed event time (ms), algorithmic flops and bytes of one GEMM kernel."""
    h = h or handle()
    n = ctypes.c_longlong(0)
    ms = ctypes.c_double(0.0)
    fl = ctypes.c_double(0.0)
    by = ctypes.c_double(0.0)
    _check("cdf_profile_end", lib().cdf_profile_end(h.ptr, GEMM_KERNELS[kernel], ctypes.byref(n), ctypes.byref(ms),
                                                    ctypes.byref(fl), ctypes.byref(by)), h.ptr)
    return {"launches": int(n.value), "total_ms": float(ms.value), "flops": float(fl.value), "bytes": float(by.value)}


# ---------------------------------------------------------------- mixed precision

def _solve_mixed(fn_name, prec, A, B, X, max_iter, info, h):
    h = h or handle(A.device)
    iters = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    n = A.shape[0]
    st = getattr(lib(), fn_name)(h.bind_stream(), UPD[prec], n, _cols(B), _p(A), _ld(A), _p(B), _ld(B), _p(X),
                                 _ld(X), int(max_iter), ctypes.byref(iters), ctypes.byref(res), _p(info))
    if st not in (CDF_OK, CDF_ERR_NOT_CONVERGED):
        _check(fn_name, st, h.ptr)
    out = {"status": st, "converged": st == CDF_OK, "iters": iters.value, "scaled_resid": res.value}
    m, f, c, p = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    sh = ctypes.c_double(0.0)
    lib().cdf_mixed_report(h.ptr, ctypes.byref(m), ctypes.byref(sh), ctypes.byref(f), ctypes.byref(c), ctypes.byref(p))
    out.update({"method": REFINE.get(m.value), "shift": sh.value, "factorizations": f.value, "corrections": c.value,
                "pcg_iterations": p.value})
    return out


def dgesv_mixed(prec: str, A, B, X, info, max_iter: int = 30, h: Handle | None = None) -> dict:
    """Mixed-precision LU + iterative refinement (see cdf_dgesv_mixed)."""
    return _solve_mixed("cdf_dgesv_mixed", prec, A, B, X, max_iter, info, h)


def dposv_mixed(prec: str, A, B, X, info, max_iter: int = 30, h: Handle | None = None) -> dict:
    """Mixed-precision Cholesky + iterative refinement (see cdf_dposv_mixed)."""
    return _solve_mixed("cdf_dposv_mixed", prec, A, B, X, max_iter, info, h)


def sgetrf_mixed(prec: str, A, W, ipiv, info, h: Handle | None = None) -> None:
    """W <- binary32 LU factors of A with a low-precision update (see cdf_sgetrf_mixed)."""
    h = h or handle(A.device)
    n = A.shape[0]
    _check("cdf_sgetrf_mixed", lib().cdf_sgetrf_mixed(h.bind_stream(), UPD[prec], n, _p(A), _ld(A), _p(W), _ld(W),
                                                      _p(ipiv), _p(info)), h.ptr)


def spotrf_mixed(prec: str, A, W, info, h: Handle | None = None) -> None:
    """lower(W) <- binary32 Cholesky factor of A with a low-precision update (see cdf_spotrf_mixed)."""
    h = h or handle(A.device)
    n = A.shape[0]
    _check("cdf_spotrf_mixed", lib().cdf_spotrf_mixed(h.bind_stream(), UPD[prec], b"L", n, _p(A), _ld(A), _p(W),
                                                      _ld(W), _p(info)), h.ptr)


def update_tile(prec: str) -> int:
    return int(lib().cdf_update_tile(UPD[prec]))


def quantize(prec: str, X: torch.Tensor, tm: int, tn: int, Q: torch.Tensor, exps: torch.Tensor,
             h: Handle | None = None) -> None:
    h = h or handle(X.device)
    m, n = X.shape[0], _cols(X)
    _check("cdf_quantize", lib().cdf_quantize(h.bind_stream(), UPD[prec], m, n, _p(X), _ld(X), tm, tn, _p(Q),
                                              _ld(Q), _p(exps)), h.ptr)


def lowp_update(prec: str, QA, ea, QB, eb, C, k: int, h: Handle | None = None) -> None:
    h = h or handle(C.device)
    m, n = C.shape[0], _cols(C)
    _check("cdf_lowp_update", lib().cdf_lowp_update(h.bind_stream(), UPD[prec], m, n, k, _p(QA), _ld(QA), _p(ea),
                                                    _p(QB), _ld(QB), _p(eb), _p(C), _ld(C)), h.ptr)


# ---------------------------------------------------------------- batched

class VBatchPlan:
    """A planned batch of small factorizations (see cdf_vbatch_plan_create)."""

    def __init__(self, sizes, kinds, dtype=F64, h: Handle | None = None, tuned: bool = True):
        """tuned: take the launch shape from the autotuner's cache entry
        nearest to the batch's largest order (if the cache has one; the
        handle's own parameters otherwise)."""
        self.h = h or handle()
        self.sizes = np.ascontiguousarray(sizes, dtype=np.int32)
        self.kinds = np.ascontiguousarray(kinds, dtype=np.int32)
        saved = {}
        self.params = {}
        if tuned and len(self.sizes):
            from . import tune as _tune
            names = _tune.SPACES["vbatch"]
            saved = {k: self.h.get_param(k) for k in names}
            self.params = _tune.apply(self.h, "vbatch", int(self.sizes.max()), "f64" if dtype == F64 else "f32")
        plan = _vp()
        try:
            st = lib().cdf_vbatch_plan_create(self.h.bind_stream(), len(self.sizes),
                                              self.sizes.ctypes.data_as(_c_int_p),
                                              self.kinds.ctypes.data_as(_c_int_p), int(dtype), ctypes.byref(plan))
        finally:
            for k, v in saved.items():
                self.h.set_param(k, v)
        _check("cdf_vbatch_plan_create", st, self.h.ptr)
        self._plan = plan

    def run(self, a_ptrs: torch.Tensor, ldas: torch.Tensor, ipiv_ptrs: torch.Tensor, infos: torch.Tensor) -> None:
        st = lib().cdf_vbatch_run(self.h.bind_stream(), self._plan, _p(a_ptrs), _p(ldas), _p(ipiv_ptrs), _p(infos))
        _check("cdf_vbatch_run", st, self.h.ptr)

    def close(self):
        if self._plan:
            lib().cdf_vbatch_plan_destroy(self._plan)
            self._plan = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def io_lower_bound_elems(kind: int, n: float, m_elems: float) -> float:
    return float(lib().cdf_io_lower_bound_elems(int(kind), float(n), float(m_elems)))


def _daap_statement(nvars, accesses, weights=None, nvertices=1.0, u=0, arrays=None) -> DaapStatement:
    """Marshal a statement: accesses = per input access, the indices of its
    distinct iteration variables (see cdf_daap_statement_t)."""
    st = DaapStatement()
    st.nvars = int(nvars)
    st.naccesses = len(accesses)
    if st.naccesses > DAAP_MAX:
        raise ValueError("too many accesses")
    for j, vs in enumerate(accesses):
        st.access_vars[j] = sum(1 << int(t) for t in set(vs))
        st.access_weight[j] = float(1.0 if weights is None else weights[j])
        st.array_id[j] = int(j if arrays is None else arrays[j])
    st.u = int(u)
    st.nvertices = float(nvertices)
    return st


def daap_chi(nvars, accesses, weights, x: float):
    """(chi(X), [|D^t|]) of one statement (see cdf_daap_chi)."""
    st = _daap_statement(nvars, accesses, weights)
    chi = ctypes.c_double()
    tile = (ctypes.c_double * DAAP_MAX)()
    _check("cdf_daap_chi", lib().cdf_daap_chi(ctypes.byref(st), float(x), ctypes.byref(chi), tile), None)
    return chi.value, list(tile[:nvars])


def daap_statement_bound(nvars, accesses, weights, nvertices, m: float, u: int = 0) -> dict:
    """The statement's I/O bound for fast memory m (see cdf_daap_statement_bound)."""
    st = _daap_statement(nvars, accesses, weights, nvertices, u)
    r = DaapResult()
    _check("cdf_daap_statement_bound", lib().cdf_daap_statement_bound(ctypes.byref(st), float(m), ctypes.byref(r)),
           None)
    return {"rho": r.rho, "x0": r.x0, "chi": r.chi, "q": r.q, "tiles": list(r.tile[:nvars]),
            "access_sizes": list(r.access[:len(accesses)])}


def daap_program_bound(statements, m: float) -> float:
    """Program bound (see cdf_daap_program_bound); statements as dicts with
    nvars, accesses, weights, nvertices, u and arrays (hashable ids)."""
    ids = {}
    arr = (DaapStatement * len(statements))()
    for i, s in enumerate(statements):
        arrays = [ids.setdefault(a, len(ids)) for a in s["arrays"]]
        arr[i] = _daap_statement(s["nvars"], s["accesses"], s["weights"], s["nvertices"], s.get("u", 0), arrays)
    q = ctypes.c_double()
    _check("cdf_daap_program_bound", lib().cdf_daap_program_bound(len(statements), arr, float(m), ctypes.byref(q)),
           None)
    return q.value
