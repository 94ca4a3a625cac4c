"""C ABI checks that run without a GPU: the library loads, exports every
function include/gpfc.h declares, and rejects bad arguments on the host
before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2312_02063_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gpfc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gpfc_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(_lib.exported_symbols())


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_and_strerror():
    lib = _lib.load()
    assert lib.gpfc_version() == 100
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.gpfc_strerror(code)
    assert lib.gpfc_strerror(-99) == b"unknown error"


def test_null_plan_and_bad_arguments_rejected_on_host():
    lib = _lib.load()
    p = ctypes.c_void_p(1)        # never dereferenced: argument checks fail first
    null = None
    assert lib.gpfc_fold(null, None, None, 10, None, 5, 64, None, None, None, None) == _lib.EINVAL
    assert lib.gpfc_fold_score(null, None, None, 0, None, 0, 64, None, None, None, None, None) == _lib.EINVAL
    assert lib.gpfc_score(null, None, None, 1, 64, 1.0, None, None, None, None, None) == _lib.EINVAL
    assert lib.gpfc_fold_naive(null, None, None, 1, None, 1, 64, None, None, None) == _lib.EINVAL
    assert lib.gpfc_plan_set_widths(null, None, 0) == _lib.EINVAL
    assert lib.gpfc_plan_create(None, 0) == _lib.EINVAL
    assert lib.gpfc_plan_destroy(null) == _lib.OK
    # negative sizes, missing pointers, nbins not a power of two, n too large
    assert lib.gpfc_fold(p, None, None, -1, None, 0, 64, None, None, None, None) == _lib.EINVAL
    assert lib.gpfc_fold(p, None, None, 5, None, 0, 64, None, None, None, None) == _lib.EINVAL
    assert lib.gpfc_fold(p, p, p, 5, None, 3, 64, None, None, None, None) == _lib.EINVAL
    assert lib.gpfc_fold(p, p, p, 5, p, 3, 0, p, p, None, None) == _lib.EINVAL
    assert lib.gpfc_fold(p, p, p, 5, p, 3, 48, p, p, None, None) == _lib.ENOTSUP
    assert lib.gpfc_fold(p, p, p, 5, p, 3, 8192, p, p, None, None) == _lib.ENOTSUP
    assert lib.gpfc_fold(p, p, p, 5, p, 3, 6144, p, p, None, None) == _lib.ENOTSUP
    assert lib.gpfc_fold(p, p, p, _lib.MAX_SAMPLES + 1, p, 3, 64, p, p, None, None) == _lib.ERANGE
    assert lib.gpfc_fold(p, p, p, 5, p, 2**31, 64, p, p, None, None) == _lib.ERANGE
    assert lib.gpfc_fold(p, p, p, 5, p, 3, 64, None, p, None, None) == _lib.EINVAL
    assert lib.gpfc_fold_score(p, p, p, 5, p, 3, 64, p, None, p, p, None) == _lib.EINVAL
    assert lib.gpfc_score(p, p, p, 3, 100, 1.0, p, p, p, p, None) == _lib.ENOTSUP
    assert lib.gpfc_score(p, p, p, 3, 8192, 1.0, p, p, p, p, None) == _lib.ENOTSUP
    assert lib.gpfc_score(p, p, p, -1, 64, 1.0, p, p, p, p, None) == _lib.EINVAL


def test_width_validation():
    lib = _lib.load()
    p = ctypes.c_void_p(1)
    arr = (ctypes.c_int32 * 4)(1, 2, 2, 3)
    assert lib.gpfc_plan_set_widths(p, arr, 4) == _lib.EINVAL        # not strictly ascending
    arr = (ctypes.c_int32 * 2)(0, 3)
    assert lib.gpfc_plan_set_widths(p, arr, 2) == _lib.EINVAL        # w < 1
    arr = (ctypes.c_int32 * 25)(*range(1, 26))
    assert lib.gpfc_plan_set_widths(p, arr, 25) == _lib.EINVAL       # too many
    arr = (ctypes.c_int32 * 2)(3, 4096)
    assert lib.gpfc_plan_set_widths(p, arr, 2) == _lib.EINVAL        # not below the largest nbins


def test_plan_options_validated_on_host():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.gpfc_plan_create_opts(None, None) == _lib.EINVAL
    assert lib.gpfc_plan_create_opts(ctypes.byref(h), None) == _lib.EINVAL
    o = _lib.PlanOpts(device=0, nw=2, split=0)
    o.widths[0], o.widths[1] = 4, 4                                    # not ascending
    assert lib.gpfc_plan_create_opts(ctypes.byref(h), ctypes.byref(o)) == _lib.EINVAL
    o = _lib.PlanOpts(device=0, nw=0, split=65)                         # split too large
    assert lib.gpfc_plan_create_opts(ctypes.byref(h), ctypes.byref(o)) == _lib.EINVAL
    o = _lib.PlanOpts(device=0, nw=0, split=0, workspace_bytes=-1)
    assert lib.gpfc_plan_create_opts(ctypes.byref(h), ctypes.byref(o)) == _lib.EINVAL
    o = _lib.PlanOpts(device=0, nw=_lib.MAX_WIDTHS + 1)
    assert lib.gpfc_plan_create_opts(ctypes.byref(h), ctypes.byref(o)) == _lib.EINVAL
    assert h.value is None


def test_batch_curves_longer_than_one_packed_pass_rejected():
    lib = _lib.load()
    p = ctypes.c_void_p(1)
    so = (ctypes.c_int64 * 3)(0, 100, 100 + _lib.MAX_PACKED + 1)
    po = (ctypes.c_int64 * 3)(0, 10, 20)
    assert lib.gpfc_batch_setup(p, so, po, 2) == _lib.ERANGE
    assert lib.gpfc_survey_setup(p, so, 2, 10, 0) == _lib.ERANGE


def test_product_path_has_no_cpu_fallback():
    # The package must not import the oracle anywhere.
    pkg = os.path.join(ROOT, "paper_2312_02063_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "gpfc_oracle" not in text, f


def test_topk_and_survey_argument_checks():
    lib = _lib.load()
    p = ctypes.c_void_p(1)
    assert lib.gpfc_topk(p, 1, 10, None, 0.0, 0, p, p, None) == _lib.EINVAL      # top < 1
    assert lib.gpfc_topk(p, 1, 10, None, 0.0, 65, p, p, None) == _lib.EINVAL     # top > 64
    assert lib.gpfc_topk(p, -1, 10, None, 0.0, 1, p, p, None) == _lib.EINVAL
    assert lib.gpfc_topk(None, 1, 10, None, 0.0, 1, p, p, None) == _lib.EINVAL
    assert lib.gpfc_topk(None, 0, 10, None, 0.0, 1, None, None, None) == _lib.OK  # nothing to do
    so = (ctypes.c_int64 * 2)(0, 10)
    assert lib.gpfc_survey_setup(None, so, 1, 10, 0) == _lib.EINVAL
    assert lib.gpfc_survey_setup(p, so, 1, -1, 0) == _lib.EINVAL
    bad = (ctypes.c_int64 * 2)(3, 10)
    assert lib.gpfc_survey_setup(p, bad, 1, 10, 0) == _lib.EINVAL
    out = _lib.SurveyOut()
    assert lib.gpfc_survey_run(None, None, p, p, p, 256, ctypes.byref(out), None) == _lib.EINVAL
    assert lib.gpfc_survey_run(p, None, p, p, p, 256, None, None) == _lib.EINVAL


def test_noalloc_arguments_rejected_on_host():
    """gpfc_fold_score_noalloc checks its arguments before any HIP call: its
    sample limit, the fused kernel's nbins range and missing pointers."""
    lib = _lib.load()
    p = ctypes.c_void_p(1)        # never dereferenced
    f = lib.gpfc_fold_score_noalloc
    assert f(p, p, -1, p, 3, 64, p, p, p, p, None) == _lib.EINVAL
    assert f(None, p, 5, p, 3, 64, p, p, p, p, None) == _lib.EINVAL
    assert f(p, p, 5, p, 3, 64, p, p, None, p, None) == _lib.EINVAL
    assert f(p, p, 5, p, 3, 0, p, p, p, p, None) == _lib.EINVAL
    assert f(p, p, 5, p, 3, 48, p, p, p, p, None) == _lib.ENOTSUP
    assert f(p, p, 5, p, 3, 512, p, p, p, p, None) == _lib.ENOTSUP
    assert f(p, p, 131073, p, 3, 64, p, p, p, p, None) == _lib.ERANGE
    assert f(p, p, 5, p, 2**31, 64, p, p, p, p, None) == _lib.ERANGE
