"""The C-ABI library loads and exports every function include/fdx.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdx_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1601_03138_amd import build, fdx
    if not os.path.exists(fdx.LIB_PATH):
        build.build()
    return ctypes.CDLL(fdx.LIB_PATH)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("fdx_create", "fdx_destroy", "fdx_set_particles", "fdx_build_tree",
                 "fdx_calc_force", "fdx_integrate", "fdx_get_forces", "fdx_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1601_03138_amd import fdx
    assert set(_declared()) <= set(fdx.EXPORTS)


def test_null_context_calls_fail_cleanly(lib):
    # argument validation happens before any device work: no GPU needed
    lib.fdx_last_error.restype = ctypes.c_char_p
    lib.fdx_last_error.argtypes = [ctypes.c_void_p]
    assert lib.fdx_last_error(None) == b"null context"
    lib.fdx_destroy.argtypes = [ctypes.c_void_p]
    assert lib.fdx_destroy(None) == 0
    lib.fdx_create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    assert lib.fdx_create(None, 0, None) == -1


def test_domain_factorisation_matches_the_oracle():
    # fdx_dd_factor is host-only logic: no GPU needed
    import oracle as O
    from paper_1601_03138_amd import fdx
    for n in range(1, 400):
        assert fdx.dd_factor(n) == O.dd_factor(n), n
    with pytest.raises(fdx.FdxError):
        fdx.dd_factor(0)
