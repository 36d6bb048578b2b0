"""The C-ABI library loads and exports every entry point declared in
include/dist.h; host-side argument checks reject bad input without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dist.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(dist_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dist_render_fwd", "dist_render_bwd", "dist_submit", "dist_poll", "dist_create",
                     "dist_destroy", "dist_saved_free", "dist_sdf_eval", "dist_sdf_vjp", "dist_last_error"):
        assert required in names


@pytest.fixture(scope="module")
def lib():
    from paper_1911_13225_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        pytest.fail("libdist.so is not built (python -m paper_1911_13225_amd.build)")
    return N.load()


def test_library_exports_every_declared_symbol(lib):
    from paper_1911_13225_amd import _native as N
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in N.EXPORTS, f"binding lacks {name}"
    assert b"gfx950" in lib.dist_version()


def test_null_arguments_are_rejected(lib):
    from paper_1911_13225_amd import _native as N
    h = ctypes.c_void_p()
    assert lib.dist_create(None, None, None, None, 0, None) == -1
    assert b"null" in lib.dist_last_error()
    assert lib.dist_render_fwd(None, None, 0, None, 0, None, 0, None, None, None, None, None, None, None, None,
                               None, None) == -1
    assert lib.dist_render_bwd(None, None, None, None, None, None, None, None, None) == -1
    assert lib.dist_saved_free(None) == -1
    assert lib.dist_destroy(None) == -1
    assert lib.dist_sdf_eval(None, None, None, None, 0, 0, 0, None, None) == -1


def test_bad_decoder_descriptions_are_rejected(lib):
    from paper_1911_13225_amd import _native as N
    h = ctypes.c_void_p()
    ptrs = (ctypes.c_void_p * 3)(1, 1, 1)
    for dims, L, skip in [((128, 128, 2), 64, -1),      # last layer not 1 wide
                          ((128, 1), 64, -1),           # too few layers
                          ((1024, 128, 1), 64, -1),     # hidden width too large
                          ((128, 128, 1), 0, -1),       # no latent
                          ((128, 128, 1), 64, 1)]:      # skip at the last hidden layer
        d = (ctypes.c_int32 * len(dims))(*dims)
        desc = N.dist_decoder_desc(len(dims), L, skip, d)
        assert lib.dist_create(ctypes.byref(h), ctypes.byref(desc), ptrs, ptrs, 0, None) == -1
