"""The C-ABI library loads and exports every function include/gavis.h
declares; host-only helpers behave (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gavis.h")


def _header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


@pytest.fixture(scope="module")
def lib():
    from paper_2605_30342_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2605_30342_amd.build import build_library
        build_library(verbose=False)
    return _lib.load()


def test_header_declares_the_three_calls():
    names = _header_functions()
    for n in ("vf_build", "vf_query_views", "select_next_view"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2605_30342_amd import _lib
    names = _header_functions()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_default_params(lib):
    from paper_2605_30342_amd import _lib
    v = _lib.default_vf_params()
    assert v.sh_degree == 2 and v.kappa == 1.0 and v.cut == 9.0 and abs(v.eps_T - 1e-4) < 1e-9
    u = _lib.default_uq_params()
    assert u.beta == 0.5 and abs(u.o0 - 0.15) < 1e-7 and u.half_logdet_Q0 == 0.0
    assert abs(u.half_logdet_Qc - 3 * __import__("math").log(0.1)) < 1e-5


def test_workspace_bytes_is_monotone(lib):
    from paper_2605_30342_amd import _lib
    p = _lib.gv_workspace()
    p.n, p.n_views, p.total_tiles, p.total_pixels, p.kind, p.sh_degree = 1000, 4, 256, 65536, 1, 2
    p.max_records, p.max_instances = 4000, 9000
    b1 = lib.gv_workspace_bytes(ctypes.byref(p))
    p.max_instances = 20000
    b2 = lib.gv_workspace_bytes(ctypes.byref(p))
    assert b2 > b1 > 0
    assert b2 - b1 >= 4 * 4 * 11000


def test_last_error_is_a_string(lib):
    assert isinstance(lib.gv_last_error(), bytes)
