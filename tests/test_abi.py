"""The C-ABI library loads and exports every entry point its header declares (CPU only)."""
import ctypes
import os
import re

import pytest

import paper_2112_06300_amd as ccd
from paper_2112_06300_amd import build as ccd_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    srcs = [os.path.join(ccd.HERE, "csrc", s) for s in ccd_build.SOURCES] + [HEADER]
    if not os.path.exists(ccd.LIB_PATH) or os.path.getmtime(ccd.LIB_PATH) < max(os.path.getmtime(s) for s in srcs):
        ccd_build.build()
    return ccd.load_library()


def test_header_declarations_are_exported(lib):
    names = _declared()
    assert set(names) == set(ccd.EXPORTED), names
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_error_string(lib):
    assert b"gfx950" in lib.ccd_version()
    assert isinstance(lib.ccd_last_error(), bytes)


def test_null_arguments_rejected_without_device(lib):
    n = ctypes.c_int64()
    st = lib.ccd_broad(None, None, None, 0, None, 0, None, 0, None, 0, ctypes.byref(n), None, 0,
                       ctypes.byref(n), None)
    assert st == ccd.CCD_ERR_INVALID_ARG
    st = lib.ccd_narrow(None, None, None, 0, None, 0, None, 0, None, 0, None, 0, 1e-6, 10, None, None,
                        None, None, None)
    assert st == ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_create(0, None) == ccd.CCD_ERR_INVALID_ARG
