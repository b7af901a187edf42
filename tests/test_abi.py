"""Host-side checks of the C ABI library (no GPU compute)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ap.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ap_status|const char\*)\s+(ap_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2505_12958_amd import ap
    L = ap.lib()
    names = declared_functions()
    assert {"ap_create", "ap_build_neighbors", "ap_eam_forces", "ap_ace_forces", "ap_blend",
            "ap_step"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ap.EXPORTS)
    assert L.ap_version().decode().startswith("ap ")


def test_create_argument_errors_without_touching_a_gpu():
    from paper_2505_12958_amd import ap
    L = ap.lib()
    h = ctypes.c_void_p()
    assert L.ap_create(None, 0, 0, None, None) == ap.AP_ERR_ARG
    assert L.ap_create(ctypes.byref(h), 0, 7, None, None) == ap.AP_ERR_ARG
    assert b"precision" in L.ap_last_error(None)
    assert L.ap_destroy(None) == ap.AP_OK


def test_null_context_is_rejected():
    from paper_2505_12958_amd import ap
    L = ap.lib()
    assert L.ap_check(None, None) == ap.AP_ERR_ARG
    assert L.ap_step(None, None, None, 1, None) == ap.AP_ERR_ARG
