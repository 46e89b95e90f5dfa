"""The C-ABI library loads, exports every entry point include/ofm.h declares,
and rejects bad arguments on the host before any device work (no GPU
needed)."""
import ctypes
import os
import re

import pytest

from paper_2305_10356_amd import ofm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ofm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ofm_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ofm.LIB_PATH):
        pytest.fail("libofm.so is not built (run __graft_entry__.build())")
    return ofm.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ofm._SIGS), "binding and header disagree"


def test_status_strings(lib):
    assert lib.ofm_status_string(0) == b"OFM_OK"
    assert lib.ofm_status_string(-3) == b"OFM_E_GRAPH"
    assert lib.ofm_status_string(-8) == b"OFM_E_UNSUPPORTED"
    assert lib.ofm_status_string(-9) == b"OFM_E_NO_ROOT"
    assert lib.ofm_status_string(-10) == b"OFM_E_UNKNOWN"
    assert lib.ofm_status_string(5) == b"OFM_E_UNKNOWN"


def test_host_argument_checks(lib):
    h = ctypes.c_void_p()
    # no output handle / empty graph / null pointers
    assert lib.ofm_build_laplacian(10, 0, None, None, None, 0, 0, None, None) == -1
    assert lib.ofm_build_laplacian(0, 0, None, None, None, 0, 0, None, ctypes.byref(h)) == -1
    assert lib.ofm_build_laplacian(10, 5, None, None, None, 0, 0, None, ctypes.byref(h)) == -1
    assert lib.ofm_build_laplacian(10, 5, ctypes.c_void_p(16), ctypes.c_void_p(16), None, 0,
                                   1 << 5, None, ctypes.byref(h)) == -1
    assert lib.ofm_build_laplacian(1 << 31, 5, ctypes.c_void_p(16), ctypes.c_void_p(16), None, 0,
                                   0, None, ctypes.byref(h)) == -2
    # weights of an unknown type are refused before anything is enqueued
    assert lib.ofm_build_laplacian(10, 5, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                   ctypes.c_void_p(16), 7, 0, None, ctypes.byref(h)) == -1
    # the root rules: bad variant, negative count, null arrays; nothing to do for 0
    assert lib.ofm_select_roots(4, 1, p16 := ctypes.c_void_p(16), p16, p16, None) == -1
    assert lib.ofm_select_roots(0, -1, p16, p16, p16, None) == -1
    assert lib.ofm_select_roots(0, 3, None, p16, p16, None) == -1
    assert lib.ofm_select_roots(1, 0, None, None, None, None) == 0
    assert lib.ofm_laplacian_destroy(None) == -1
    assert lib.ofm_laplacian_upper(None, None, None) == -1
    assert lib.ofm_workspace_destroy(None) == -1
    opts = ofm.Opts(0, 1, 10, 1, 0, 0, 0.0, 0.0)
    assert lib.ofm_workspace_create(None, 8, ctypes.byref(opts), ctypes.byref(h)) == -1
    # the options struct of the binding has the header's layout
    assert ctypes.sizeof(ofm.Opts) == 64 and ofm.Opts.freeze_eps.offset == 56
    assert lib.ofm_init(None, None, None) == -1
    assert lib.ofm_step(None, None, None) == -1
    assert lib.ofm_apply_A(None, 8, 1, None, None, None) == -1
    # shapes
    p = ctypes.c_void_p(16)
    assert lib.ofm_row_normalize(10, 65, 1, p, p, None) == -2
    assert lib.ofm_row_normalize(10, 4, 7, p, p, None) == -1
    assert lib.ofm_row_normalize(0, 4, 1, p, p, None) == 0
    assert lib.ofm_kmeans_assign(10, 0, 3, p, p, p, None, None) == -2
    assert lib.ofm_kmeans_assign(10, 4, 2000, p, p, p, None, None) == -2
    assert lib.ofm_kmeans_assign(0, 4, 3, p, p, p, None, None) == 0
    u = (ctypes.c_double * 2)(0.5, 1.5)
    assert lib.ofm_kmeans(10, 4, 2, p, u, 10, p, p, None, None) == -1
    assert lib.ofm_kmeans(10, 4, 20, p, u, 10, p, p, None, None) == -2
