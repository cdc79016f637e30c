"""The C-ABI library loads and exports every symbol include/ddelm.h declares.

No compute call is made, so this runs without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddelm.h")
LIB = os.path.join(ROOT, "paper_2503_10032_amd", "libddelm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddelm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libddelm.so not built: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("ddelm_setup", "ddelm_factor", "ddelm_solve", "ddelm_evaluate", "ddelm_destroy", "ddelm_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_2503_10032_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_default_options_without_gpu(lib):
    from paper_2503_10032_amd import _lib
    l = _lib.load()
    o = _lib.Options()
    l.ddelm_default_options(ctypes.byref(o))
    assert o.theta == 0.999 and o.coarse == 2 and o.precision == 0 and o.max_nrhs == 1
    # the defaults the header documents
    assert (o.tol, o.maxit, o.cg_mode) == (1e-8, 20000, 0)
    assert (o.refine_maxit, o.refine_tol, o.inner_tol) == (10, 1e-9, 1e-3)


def test_setup_rejects_null_problem(lib):
    from paper_2503_10032_amd import _lib
    l = _lib.load()
    ctx = ctypes.c_void_p()
    assert l.ddelm_setup(ctypes.byref(ctx), None, None, None) == -1
