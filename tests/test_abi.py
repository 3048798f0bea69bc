"""The C ABI library loads and exports every entry point the header declares.

CPU only: nothing here launches a kernel.  Argument validation that happens
before any device call is exercised too.
"""
import ctypes
import os
import re

import pytest

from paper_2002_01108_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "aao.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aao_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2002_01108_amd import build
        build.build(verbose=False)
    return binding.load()


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("aao_setup", "aao_apply_A", "aao_apply_Pinv", "aao_solve", "aao_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) == set(binding.SIGNATURES)


def test_status_strings(lib):
    assert lib.aao_status_string(0) == b"AAO_OK"
    assert lib.aao_status_string(-1) == b"AAO_EINVAL"
    assert lib.aao_status_string(1) == b"AAO_NOT_CONVERGED"


@pytest.mark.parametrize("args", [
    (2, 15, 15, 1, 16, 1.0, 0.0),      # eps = 0 (Theorem 3.1 needs eps in (0,1])
    (2, 15, 15, 1, 16, 1.0, 1.5),      # eps > 1
    (2, 15, 15, 1, 16, 1.0, -0.1),
    (2, 15, 15, 1, 12, 1.0, 0.1),      # n not a power of two
    (2, 15, 15, 1, 1, 1.0, 0.1),       # n < 2
    (2, 15, 15, 1, 2048, 1.0, 0.1),    # n too large
    (4, 15, 15, 15, 16, 1.0, 0.1),     # dim
    (2, 0, 15, 1, 16, 1.0, 0.1),       # empty grid
    (2, 15, 2000, 1, 16, 1.0, 0.1),    # grid too large
    (1, 15, 1, 1, 16, 0.0, 0.1),       # T = 0
    (1, 15, 1, 1, 16, float("nan"), 0.1),
    (1, 15, 1, 1, 16, 1.0, float("nan")),
])
def test_setup_rejects_bad_arguments(lib, args):
    h = ctypes.c_void_p()
    st = lib.aao_setup(*args, ctypes.byref(h))
    assert st == binding.EINVAL
    assert not h.value


def test_null_context_is_rejected(lib):
    assert lib.aao_apply_A(None, None, None) == binding.EINVAL
    assert lib.aao_apply_Pinv(None, None, None) == binding.EINVAL
    assert lib.aao_sync(None) == binding.EINVAL
    lib.aao_destroy(None)


def test_every_context_entry_point_rejects_null(lib):
    """Each entry point that takes a context returns EINVAL for a null one
    before it touches the device (other arguments: null pointers, ones)."""
    skip = {"aao_destroy", "aao_last_error"}
    checked = 0
    for name, (res, args) in binding.SIGNATURES.items():
        if name in skip or not args or args[0] is not ctypes.c_void_p or res is not ctypes.c_int:
            continue
        vals = [None]
        for t in args[1:]:
            if t in (ctypes.c_int,):
                vals.append(1)
            elif t in (ctypes.c_double, ctypes.c_float):
                vals.append(1.0)
            else:
                vals.append(None)
        assert getattr(lib, name)(*vals) == binding.EINVAL, name
        checked += 1
    assert checked >= 27
