"""The C ABI library loads and exports every entry point the header declares (no GPU calls)."""

import ctypes
import os
import subprocess

import pytest

import paper_1706_00692_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(pk.library_path()):
        pytest.skip("libifeast.so not built")
    return pk.load_library()


def test_header_declares_the_boundary():
    names = pk.exported_symbols()
    for must in ("ifeast_create", "ifeast_destroy", "ifeast_solve", "ifeast_solve_resident", "ifeast_solve_dev",
                 "ifeast_footprint",
                 "ifeast_submit", "ifeast_poll", "ifeast_wait", "ifeast_spmm_shifted_dev", "ifeast_filter_dev",
                 "ifeast_rayleigh_ritz_dev", "ifeast_matrix_create", "ifeast_status_str", "ifeast_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib_or_skip()
    out = subprocess.run(["nm", "-D", "--defined-only", pk.library_path()], capture_output=True, text=True).stdout
    defined = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in pk.exported_symbols():
        assert name in defined, name
        assert hasattr(lib, name)


def test_status_strings_and_version():
    lib = _lib_or_skip()
    assert lib.ifeast_status_str(0) == b"ok"
    assert b"invalid" in lib.ifeast_status_str(-1)
    assert b"gfx950" in lib.ifeast_version()


def test_footprint_host_only():
    _lib_or_skip()
    c = {"kind": "half", "emin": 0.5, "emax": 0.8, "rule": "gl", "nc": 8}
    p = pk.params_struct(16, max_inner=4)
    b1 = pk.footprint(400, 1920, 0, c, p)
    b2 = pk.footprint(800, 3840, 0, c, p)
    assert 0 < b1 < b2
    # mixed precision halves the basis
    big = pk.footprint(262144, 1810432, 0, dict(c, nc=8), pk.params_struct(80, max_inner=8))
    bigm = pk.footprint(262144, 1810432, 0, dict(c, nc=8), pk.params_struct(80, max_inner=8, precision=pk.PREC_MIXED))
    assert bigm < big and big > 20e9
    with pytest.raises(pk.IFeastError):
        pk.footprint(400, 1920, 0, c, pk.params_struct(20))  # m0 not a multiple of 16
    with pytest.raises(pk.IFeastError):
        pk.footprint(400, 1920, 0, dict(c, emin=1.0, emax=0.5), p)


def test_library_has_gfx950_code_object():
    _lib_or_skip()
    blob = open(pk.library_path(), "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob
