"""The C ABI: every function declared in include/rcurves.h is exported by the
built library, and host-side argument validation (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rcurves.h")
LIB = os.path.join(ROOT, "paper_2006_07859_amd", "librcurves.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("rc_create", "rc_energy", "rc_differential", "rc_sobolev_apply", "rc_sobolev_gradient",
              "rc_line_search_step", "rc_step", "rc_bh_differential"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_the_header():
    from paper_2006_07859_amd import _lib

    assert sorted(_lib.EXPORTED) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_argument_validation_without_gpu():
    from paper_2006_07859_amd import _lib

    lib = _lib.load()
    o = _lib.SolveOpts()
    lib.rc_default_solve_opts(ctypes.byref(o))
    assert o.solver == _lib.RC_SOLVE_PCG_MG and o.tol == 1e-6
    h = ctypes.c_void_p()
    e = (ctypes.c_int32 * 8)(0, 1, 1, 2, 2, 3, 3, 0)
    # alpha <= 1 and beta outside [alpha + 2, 2 alpha + 1) are rejected before any device work
    assert lib.rc_create(4, 4, e, 1.0, 4.0, 1, None, ctypes.byref(h)) == 2
    assert lib.rc_create(4, 4, e, 2.0, 3.5, 1, None, ctypes.byref(h)) == 2
    assert lib.rc_create(4, 4, e, 2.0, 5.0, 1, None, ctypes.byref(h)) == 2
    # bad sizes, endpoints and dtype
    assert lib.rc_create(0, 4, e, 2.0, 4.0, 1, None, ctypes.byref(h)) == 1
    bad = (ctypes.c_int32 * 8)(0, 1, 1, 2, 2, 7, 3, 0)
    assert lib.rc_create(4, 4, bad, 2.0, 4.0, 1, None, ctypes.byref(h)) == 1
    loop = (ctypes.c_int32 * 8)(0, 1, 1, 1, 2, 3, 3, 0)
    assert lib.rc_create(4, 4, loop, 2.0, 4.0, 1, None, ctypes.byref(h)) == 3
    assert lib.rc_create(4, 4, e, 2.0, 4.0, 7, None, ctypes.byref(h)) == 1
    assert b"alpha" in lib.rc_last_error() or len(lib.rc_last_error()) > 0
    # null context
    assert lib.rc_energy(None, None, None) == 1
    assert lib.rc_sync_status(None, None) == 1
