"""The allocation-free LU entry point (cdf_dgetrf_noalloc), through the C ABI.

Its output is held to the existing entry point's: cdf_dgetrf with U12 solved
in place (CDF_PARAM_LU_U12 = 1) runs the same kernels in the same order, so
pivots and factors must agree bit for bit; both are also held to the oracle
(identical pivots, rounding-order tolerance, backward error <= 10).  Two calls
in a row, the second smaller, on a handle whose workspace stays empty.
"""
import ctypes

import numpy as np
import pytest

import workloads
from tests import gpu_util

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2108_09337_amd as cdf  # noqa: E402


def _existing_entry(a):
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = cdf.handle()
        h.set_param("lu_u12", 1)
        A = cdf.to_device(a)
        n = a.shape[0]
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        cdf.dgetrf(A, ipiv, info, h)
        torch.cuda.synchronize()
        h.set_param("lu_u12", 0)
        return cdf.to_host(A), ipiv.cpu().numpy(), int(info.item())


def test_noalloc_lu_two_calls_match_existing_entry(oracle_mod):
    L = cdf.lib()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h = cdf.Handle()  # a handle of its own: its workspace starts (and must stay) empty
        for n, seed in ((1300, 11), (700, 12)):
            a = workloads.lu_uniform(n, seed=seed)
            A = cdf.to_device(a)
            ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
            info = torch.full((1,), -7, dtype=torch.int32, device="cuda")
            print(f"cdf_dgetrf_noalloc n={n} seed={seed}", flush=True)
            st = L.cdf_dgetrf_noalloc(h.bind_stream(), n, ctypes.c_void_p(A.data_ptr()), A.stride(1),
                                      ctypes.c_void_p(ipiv.data_ptr()), ctypes.c_void_p(info.data_ptr()))
            assert st == cdf.CDF_OK
            assert L.cdf_device_status(h.ptr) == cdf.CDF_OK
            assert h.workspace_bytes() == 0, "the allocation-free entry point grew the workspace"
            lu, ip, inf = cdf.to_host(A), ipiv.cpu().numpy(), int(info.item())
            lu_e, ip_e, inf_e = _existing_entry(a)
            assert inf == inf_e == 0
            assert np.array_equal(ip, ip_e)
            assert np.array_equal(lu, lu_e), float(np.max(np.abs(lu - lu_e)))
            lu_or, ip_or, _ = oracle_mod.dgetrf(a)
            assert np.array_equal(ip, ip_or)
            tol = gpu_util.lu_parity_tolerance(lu_or)
            assert np.all(np.abs(lu - lu_or) <= tol)
            assert oracle_mod.lu_backward_error(a, lu, ip) <= 10.0
        h.close()


def test_noalloc_lu_rejects_oversize():
    L = cdf.lib()
    h = cdf.handle()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = L.cdf_dgetrf_noalloc(h.bind_stream(), 131073, None, 131073, None, ctypes.c_void_p(info.data_ptr()))
    assert st == cdf.CDF_ERR_INVALID_ARG and L.cdf_last_bad_arg(h.ptr) == 2
