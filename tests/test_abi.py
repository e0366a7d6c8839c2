"""The C-ABI library loads and exports every entry point include/sesm.h
declares (no GPU needed; no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sesm.h")
LIB = os.path.join(ROOT, "paper_1707_04950_amd", "libsesm.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"SESM_API\s+[\w\s\*]+?\b(sesm_\w+)\s*\(", src)))


def test_header_declares_api():
    names = declared()
    for n in ("sesm_create", "sesm_destroy", "sesm_set_surface", "sesm_matvec", "sesm_matvec_batch", "sesm_rhs",
              "sesm_solve", "sesm_efficiencies", "sesm_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsesm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsesm.so not built")
def test_null_context_is_rejected_without_gpu_work():
    import paper_1707_04950_amd as m
    lib = m.load_library()
    assert lib.sesm_set_surface(None, None, 1.0, 1.0, 0.0, 0, 1.0, None) == m.SESM_EINVAL
    assert lib.sesm_matvec(None, None, None) == m.SESM_EINVAL
    assert lib.sesm_matvec_batch(None, 1, None, 1, None, 1) == m.SESM_EINVAL
    assert lib.sesm_solve(None, None, None, 1e-10, 10, 0, 0, None) == m.SESM_EINVAL
    assert lib.sesm_timing_enable(None, 0, 1) == m.SESM_EINVAL
    assert lib.sesm_timing_read(None, None, 0) == m.SESM_EINVAL
    assert lib.sesm_last_error(None) == b"null context"
    assert lib.sesm_destroy(None) == m.SESM_OK
