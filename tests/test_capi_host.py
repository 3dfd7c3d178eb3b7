"""Host-side checks of the C ABI library (no GPU): it loads, exports every function the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abgmres.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2110_01481_amd as abg
    if not os.path.exists(abg.LIB_PATH):
        from paper_2110_01481_amd.build import build
        build()
    return abg.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("abg_create_geometry", "abg_fp_apply", "abg_bp_apply", "abg_ab_gmres",
                     "abg_ba_gmres"):
        assert required in names


def test_every_declared_function_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    import paper_2110_01481_amd as abg
    assert sorted(abg.EXPORTS) == declared_functions()


def test_invalid_geometry_rejected_without_device(lib):
    h = ctypes.c_void_p()
    EINVAL = -1
    assert lib.abg_create_geometry(0, 10, 0.0, 180.0, None, 11, 1.0, ctypes.byref(h)) == EINVAL
    assert lib.abg_create_geometry(16, 0, 0.0, 180.0, None, 11, 1.0, ctypes.byref(h)) == EINVAL
    assert lib.abg_create_geometry(16, 10, 0.0, 180.0, None, 0, 1.0, ctypes.byref(h)) == EINVAL
    assert lib.abg_create_geometry(16, 10, 0.0, 180.0, None, 11, 0.5, ctypes.byref(h)) == EINVAL
    assert lib.abg_create_geometry(16, 10, 0.0, float("nan"), None, 11, 1.0, ctypes.byref(h)) == EINVAL
    assert lib.abg_create_geometry(16, 10, 0.0, 180.0, None, 11, 1.0, None) == EINVAL
    assert lib.abg_fp_apply(None, 1, None, None, None, 0, None) == EINVAL
    assert lib.abg_bp_apply(None, 0, 1, None, None, None) == EINVAL
    assert lib.abg_destroy_geometry(None) == 0


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, 1, 2, 3):
        s = lib.abg_status_string(code)
        assert s and s != b"unknown status"
    assert lib.abg_status_string(99) == b"unknown status"
