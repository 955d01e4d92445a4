"""The C-ABI library loads and exports every symbol the header declares (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2108_09337_amd", "libcdnafact.so")
HEADER = os.path.join(ROOT, "include", "cdnafact.h")


def _declared():
    text = open(HEADER).read()
    decl = set(re.findall(r"^\s*(?:CDF_API\s+)?[A-Za-z_][\w\s\*]*?\b(cdf_\w+)\s*\(", text, flags=re.M))
    exported = set(re.findall(r"^CDF_API\s+[\w\s\*]+?\b(cdf_\w+)\s*\(", text, flags=re.M))
    assert decl == exported, f"declared without CDF_API: {sorted(decl - exported)}"
    return sorted(decl)


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("cdf_dgetrf", "cdf_dgetrs", "cdf_dpotrf", "cdf_dpotrs", "cdf_dgesv_mixed", "cdf_dposv_mixed",
                 "cdf_vbatch_plan_create", "cdf_vbatch_run", "cdf_vbatch_plan_destroy",
                 "cdf_io_lower_bound_elems", "cdf_quantize", "cdf_lowp_update", "cdf_dgemm_update"):
        assert need in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcdnafact.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcdnafact.so not built")
def test_io_bound_host_function_matches_oracle(oracle_mod):
    lib = ctypes.CDLL(LIB)
    f = lib.cdf_io_lower_bound_elems
    f.restype = ctypes.c_double
    f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
    for kind in (0, 1):
        for n, m in ((10, 100), (32768, 20480), (65536, 86016)):
            assert f(kind, n, m) == pytest.approx(oracle_mod.io_lower_bound_elems(kind, n, m), rel=1e-14)
    assert f(2, 10, 10) < 0 and f(0, 10, 0) < 0


def test_oracle_and_library_share_no_code():
    """The oracle is C compiled by gcc from oracle/; the library is HIP from the
    package's csrc/.  Neither source tree includes or names the other."""
    csrc = os.path.join(ROOT, "paper_2108_09337_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower(), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".py")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "cdnafact" not in text and "paper_2108_09337_amd" not in text, f
