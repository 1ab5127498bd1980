"""The C ABI library loads without a GPU and exports what include/hough.h declares."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hough.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1311_2769_amd import hough
    if not os.path.exists(hough.LIB_PATH):
        from paper_1311_2769_amd import build
        build.build()
    return hough.load()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(hough_\w+)\s*\(", text, re.M)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for s in ("hough_ctx_create", "hough_vote", "hough_peaks", "hough_event_batch"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_binding_covers_the_header():
    from paper_1311_2769_amd import hough
    assert sorted(hough.SYMBOLS) == declared_symbols()


def test_status_strings(lib):
    assert lib.hough_status_str(0) == b"ok"
    assert lib.hough_status_str(-1) == b"invalid argument"
    assert lib.hough_status_str(-3) == b"HIP runtime error"
    assert lib.hough_version().startswith(b"hough-mi355x")


def test_null_context_is_rejected_without_touching_the_device(lib):
    EINVAL = -1
    nul = None
    assert lib.hough_vote(nul, nul, nul, 0, nul, nul, nul) == EINVAL
    assert lib.hough_peaks(nul, nul, 1, nul, 0, nul, nul) == EINVAL
    assert lib.hough_event_batch(nul, 1, nul, nul, nul, 1, nul, nul, nul, nul, nul, nul) == EINVAL
    assert lib.hough_set_launch(nul, 0, 8, 256, 1) == EINVAL
    assert lib.hough_associate(nul, nul, nul, 0, nul, nul, 0, 1, nul, 0, nul, nul) == EINVAL
    from paper_1311_2769_amd.hough import _Grid
    out = ctypes.c_void_p()
    assert lib.hough_ctx_create(None, None, None) == EINVAL
    g = _Grid(1, 2, 8, -1.0, 4.0, 1, 1, None, 0)            # n_phi < 3
    assert lib.hough_ctx_create(ctypes.byref(out), ctypes.byref(g), None) == EINVAL
    g = _Grid(4, 8, 8, -1.0, 4.0, 1, 1, None, 0)            # 3D grid without a d0 table
    assert lib.hough_ctx_create(ctypes.byref(out), ctypes.byref(g), None) == EINVAL
    g = _Grid(1, 8, 7, -1.0, 4.0, 1, 1, None, 1)            # u16 with odd n_kappa
    assert lib.hough_ctx_create(ctypes.byref(out), ctypes.byref(g), None) == EINVAL
    g = _Grid(1, 8, 8, -1.0, 4.0, None, 1, None, 0)         # missing table
    assert lib.hough_ctx_create(ctypes.byref(out), ctypes.byref(g), None) == EINVAL
    g = _Grid(1, 8, 8, -1.0, 4.0, 1, 1, None, 0, 7)         # unknown track family
    assert lib.hough_ctx_create(ctypes.byref(out), ctypes.byref(g), None) == EINVAL
    g = _Grid(2, 8, 8, -1.0, 4.0, 1, 1, 1, 0, 1)            # straight lines have no d0 axis of their own
    assert lib.hough_ctx_create(ctypes.byref(out), ctypes.byref(g), None) == EINVAL
    g = _Grid(1, 8, 8, -1.0, 4.0, 1, 1, None, 0, 0, 2)      # forward option is 0 or 1
    assert lib.hough_ctx_create(ctypes.byref(out), ctypes.byref(g), None) == EINVAL
    from paper_1311_2769_amd.hough import _Opts
    tab = (ctypes.c_float * 8)()
    g = _Grid(1, 8, 8, -1.0, 4.0, ctypes.addressof(tab), ctypes.addressof(tab), None, 0)
    for o in (_Opts(1, -1, None), _Opts(-1, 10, None), _Opts(1, (1 << 30) + 1, None)):
        assert lib.hough_ctx_create(ctypes.byref(out), ctypes.byref(g), ctypes.byref(o)) == EINVAL


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1311_2769_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "hough_oracle" not in text, f
