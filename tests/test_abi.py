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
    srcs = [os.path.join(ccd.HERE, "csrc", s) for s in ccd_build.SOURCES + ccd_build.HEADERS] + [HEADER]
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


def test_new_entry_points_reject_null_arguments_without_device(lib):
    P = ctypes.c_void_p
    out = P()
    n = ctypes.c_int64()
    # batches
    offs = (ctypes.c_int64 * 2)(0, 0)
    assert lib.ccd_batch_create(None, 1, offs, offs, offs, 0, 0, ctypes.byref(out)) == ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_batch_run(None, None, None, None, None, 1e-6, 10, None, None, ctypes.byref(n), ctypes.byref(n),
                             None, None, None, None, 0, None) == ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_batch_autotune(None, None, None, None, None, 1e-6, 10, None, None, None, None, None, None, None,
                                  None) == ccd.CCD_ERR_INVALID_ARG
    lib.ccd_batch_destroy(None)  # no-op
    # tuning
    t = ccd.Tuning(16, 0, 1024, 13, 0, 256, 1)
    assert lib.ccd_set_tuning(None, ctypes.byref(t)) == ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_get_tuning(None, ctypes.byref(t)) == ccd.CCD_ERR_INVALID_ARG
    # learned schedule pieces
    assert lib.ccd_mlp_predict(None, None, None, None, 0, None, None) == ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_mlp_grad(None, None, None, None, None, 0, None, None, None) == ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_adam_step(None, None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == \
        ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_features(None, None, None, 0, None, 0, None, 0, None, 0, None, 0, 1e-6, None, None) == \
        ccd.CCD_ERR_INVALID_ARG
    sch = ccd.Schedule(ccd.SCHED_PLAIN, None, None, None, 0.0, 0)
    assert lib.ccd_narrow_sched(None, None, None, 0, None, 0, None, 0, None, 0, None, 0, 1e-6, 10, None, None, None,
                                None, ctypes.byref(sch), None) == ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_detect(None, None, None, 0, None, 0, None, 0, None, 0, ctypes.byref(n), None, 0, ctypes.byref(n),
                          1e-6, 10, None, None, None, None, None, None) == ccd.CCD_ERR_INVALID_ARG
    assert lib.ccd_last_error()  # a message is left


def test_model_parameter_count_matches_header():
    text = open(HEADER).read()
    assert f"#define CCD_MODEL_PARAMS {ccd.MODEL_PARAMS}" in text
    assert f"#define CCD_NUM_FEATURES {ccd.NUM_FEATURES}" in text
    assert ccd.MODEL_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def test_binding_rejects_bad_tensors_before_any_call():
    """Tensors passed as raw pointers are checked for dtype, device, contiguity and size first (a CPU
    tensor, a float32 V0, a transposed view or a short output would otherwise be read or written out of
    bounds by the kernels)."""
    torch = pytest.importorskip("torch")
    V = torch.zeros((4, 3), dtype=torch.float64)
    with pytest.raises(ValueError, match="cuda"):
        ccd._require(V, "V0", torch.float64, 0, cols=3)
    with pytest.raises(ValueError, match="dtype"):
        ccd._require(V.float(), "V0", torch.float64, 0, cols=3)
    with pytest.raises(ValueError, match="dtype"):
        ccd._require(torch.zeros((4, 2), dtype=torch.int64), "E", torch.int32, 0, cols=2)
    with pytest.raises(ValueError):
        ccd._require([1.0, 2.0], "V0", torch.float64, 0)
