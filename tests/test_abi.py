"""The C-ABI library loads and exports every symbol the header declares.
CPU only: no computation is requested."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gp_ssm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_ssm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("gp_ssm_loglik", "gp_ssm_loglik_grad", "gp_ssm_smooth", "gp_ssm_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2601_02527_amd as gp
    if not os.path.exists(gp.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(gp.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(gp.EXPORTS) == declared_functions()


def test_version_and_error_string():
    import paper_2601_02527_amd as gp
    if not os.path.exists(gp.LIB_PATH):
        pytest.skip("library not built")
    L = gp.library()
    assert b"gfx950" in L.gp_ssm_version()
    assert isinstance(L.gp_ssm_last_error(), bytes)


def test_argument_validation_precedes_device_work():
    """Invalid arguments are rejected before the library looks for a device."""
    import paper_2601_02527_amd as gp
    if not os.path.exists(gp.LIB_PATH):
        pytest.skip("library not built")
    L = gp.library()
    h = ctypes.c_void_p()
    rc = L.gp_ssm_plan_create(0, None, None, None, None, None, None, None, ctypes.byref(h))
    assert rc == -1 and not h.value
    rc = L.gp_ssm_plan_create(1, None, None, None, None, None, None, None, ctypes.byref(h))
    assert rc == -1
    rc = L.gp_ssm_plan_loglik(None, 1, None, None, None, None, None, None, None)
    assert rc == -1
