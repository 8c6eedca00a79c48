"""The C-ABI library loads and exports every symbol include/qtx.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1903_00548_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "qtx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qtx_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for n in ("qtx_create", "qtx_destroy", "qtx_set_lead", "qtx_set_device", "qtx_set_potential",
              "qtx_solve", "qtx_solve_device", "qtx_solve_batch", "qtx_problem_create",
              "qtx_self_energy", "qtx_charge", "qtx_last_error", "qtx_set_stream"):
        assert n in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libqtx.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(_lib.LIB_PATH)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    assert set(header_functions()) <= set(_lib._SIGS)


def test_info_struct_layout_matches_header():
    assert ctypes.sizeof(_lib.qtx_info) == 24
    assert _lib.INFO_DTYPE.itemsize == 24


def test_version_string(lib):
    lib.qtx_version.restype = ctypes.c_char_p
    assert b"qtx" in lib.qtx_version()


def test_null_arguments_rejected_without_device(lib):
    lib.qtx_create.argtypes = [ctypes.c_int, ctypes.c_void_p]
    assert lib.qtx_create(0, None) == _lib.EINVAL
    lib.qtx_charge.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int] * 0 + []
    # qtx_charge with NULL pointers is pure host code
    f = lib.qtx_charge
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    assert f(None, None, 1, 1, None, 0.0, 0.0, 0.025, None) == _lib.EINVAL


def test_charge_helper_matches_its_definition(lib):
    """qtx_charge is host code: charge_i = sum_k w_k (f_L n^L_ik + f_R n^R_ik)."""
    f = lib.qtx_charge
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    import numpy as np
    from oracle import integrals as oint
    rng = np.random.default_rng(3)
    nE, N = 17, 5
    E = np.sort(rng.uniform(-1, 1, nE))
    w = rng.uniform(0, 0.1, nE)
    ldos = rng.uniform(0, 3, (nE, 2, N))
    out = np.zeros(N)
    muL, muR, kT = 0.12, -0.05, 0.03
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert f(p(ldos), p(w), nE, N, p(E), muL, muR, kT, p(out)) == _lib.OK
    ref = (w * oint.fermi(E, muL, kT)) @ ldos[:, 0, :] + (w * oint.fermi(E, muR, kT)) @ ldos[:, 1, :]
    assert np.abs(out - ref).max() < 1e-13
    assert f(p(ldos), p(w), nE, N, p(E), muL, muR, 0.0, p(out)) == _lib.EINVAL       # kT must be > 0


def test_every_option_is_documented_in_the_header():
    """Every name qtx_set_option accepts appears in the header's option
    table (quoted), and every quoted name in that table is accepted."""
    src = open(os.path.join(ROOT, "paper_1903_00548_amd", "csrc", "qtx_api.cpp")).read()
    hdr = open(os.path.join(ROOT, "include", "qtx.h")).read()
    accepted = set(re.findall(r'n == "([a-z_]+)"', src))
    table = hdr[hdr.index("Tuning parameters of a context"):]
    table = table[:table.index("qtx_status qtx_set_option")]
    documented = set(re.findall(r'\*\s+"([a-z_]+)"', table))
    assert accepted, "no option names found in qtx_api.cpp"
    assert accepted == documented, (sorted(accepted - documented), sorted(documented - accepted))
