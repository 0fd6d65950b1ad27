"""The C-ABI library loads, exports every symbol include/algdist.h declares,
and rejects bad arguments on the host -- all without a GPU (no compute)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "algdist.h")
LIB = os.path.join(ROOT, "paper_1106_5990_amd", "libalgdist.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\b([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "switch", "return")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1106_5990_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_path():
    names = declared_functions()
    for n in ("setup_testvectors", "algebraic_distance", "strength_graph", "ls_interp",
              "algdist_create", "algdist_destroy", "algdist_status", "algdist_last_error",
              "csr_validate"):
        assert n in names, n


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), "missing export %s" % n
    lib.algdist_version.restype = C.c_int
    assert lib.algdist_version() == 1


def test_host_side_rejections_without_device(lib):
    """Null handles and pointers are refused before any device call."""
    lib.setup_testvectors.restype = C.c_int
    lib.algebraic_distance.restype = C.c_int
    lib.ls_interp.restype = C.c_int
    lib.algdist_create.restype = C.c_int
    assert lib.algdist_create(None, 0) == 1  # AD_EINVAL
    assert lib.setup_testvectors(None, None, 8, C.c_uint64(0), None, 0, 1, C.c_double(0.5), None, 0,
                                 None, None, 0, None) == 1
    assert lib.algebraic_distance(None, None, 8, None, None, 0, None, None, C.c_double(0), None,
                                  None, None, None) == 1
    assert lib.ls_interp(None, None, 8, None, None, None, None, 4, 0, None, None, None, None,
                         None, None) == 1
