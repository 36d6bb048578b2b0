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


def test_eps_helper_reproduces_the_paper_example(lib):
    """App. A.2: f = 60 mm, d_min = 10 cm, S = 32 mm, R = 512 give eps of about
    0.5e-4 m, and neighbouring pixels' points about 1e-4 m = 2 eps apart
    (Sec. 3.2); cos^2 scaling off the optical axis."""
    import math
    from conftest import load_golden
    from paper_1911_13225_amd import api
    g = load_golden("worked_examples.txt")
    e = api.dist_eps_for_camera(g["eps.dmin_m"], g["eps.sensor_m"], g["eps.focal_m"], int(g["eps.res"]))
    assert abs(e - g["eps.approx_m"]) / g["eps.approx_m"] < 0.05
    assert abs(2 * e - g["spacing.approx_m"]) / g["spacing.approx_m"] < 0.05
    e30 = api.dist_eps_for_camera(g["eps.dmin_m"], g["eps.sensor_m"], g["eps.focal_m"], int(g["eps.res"]),
                                  math.radians(30))
    assert abs(e30 / e - math.cos(math.radians(30)) ** 2) < 1e-12
    out = ctypes.c_double()
    assert lib.dist_eps_for_camera(0.0, 1.0, 1.0, 1, 0.0, ctypes.byref(out)) == -1
    assert lib.dist_eps_for_camera(1.0, 1.0, 1.0, 0, 0.0, ctypes.byref(out)) == -1


def test_loss_and_adam_reject_bad_arguments_on_the_host(lib):
    assert lib.dist_render_loss(0, 4, 4, None, None, None, None, None, None, 1.0, 1.0, 0.0, None, None, None,
                                None, None) == -1
    assert lib.dist_render_loss(1, 4, 4, None, None, None, None, None, None, 1.0, 1.0, 0.0, None, None, None,
                                None, None) == -1
    assert lib.dist_adam_step(None, None, None, None, 4, 1e-2, 0.9, 0.999, 1e-8, 1, None) == -1
