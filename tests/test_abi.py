"""CPU checks of the C ABI: the library loads, exports every function that
include/mgs.h declares, and rejects bad arguments on the host (no kernel runs)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgs_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2603_11531_amd import _lib
    return _lib.lib()


def test_header_declares_the_scope_entry_points():
    names = declared_functions()
    for required in ("mgs_enhance", "mgs_project", "mgs_bin", "mgs_blend_oit", "mgs_render_backward",
                     "mgs_bin_sorted", "mgs_blend_sorted"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_error_string(lib):
    assert lib.mgs_version().decode().startswith("mgs")
    assert isinstance(lib.mgs_last_error().decode(), str)


def test_host_side_validation(lib):
    from paper_2603_11531_amd import _lib as L
    nb = C.c_size_t()
    assert lib.mgs_bin_workspace(100, 4, 4, 1000, C.byref(nb)) == L.MGS_OK and nb.value > 0
    assert lib.mgs_bin_workspace(-1, 4, 4, 1000, C.byref(nb)) == L.MGS_ERR_INVALID_ARG
    # supertile ids share a 32-bit key with a 12-bit tile rectangle: at most 2^20 - 1 supertiles
    # of 8x8 tiles (65535 tiles across = 8192 supertiles; 8192 x 128 = 2^20 is the first grid over)
    assert lib.mgs_bin_workspace(100, 65535, 8 * 128, 1000, C.byref(nb)) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_bin_workspace(100, 65535, 8 * 127, 1000, C.byref(nb)) == L.MGS_OK
    pz = L.mgs_projected()
    assert lib.mgs_bin(C.byref(pz), 0, 65535, 8 * 128, None, 0, None, None, 0, None, None) == L.MGS_ERR_INVALID_ARG
    assert "supertiles" in lib.mgs_last_error().decode()
    assert lib.mgs_batch_workspace(1000, (1 << 20) - 1, 1000, C.byref(nb)) == L.MGS_OK
    # the split blend's work items hold a 24-bit tile id
    assert lib.mgs_blend_oit_split_workspace(4096, 4095, 1000, C.byref(nb)) == L.MGS_OK
    assert lib.mgs_blend_oit_split_workspace(4096, 4096, 1000, C.byref(nb)) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_batch_workspace(1000, 1 << 20, 1000, C.byref(nb)) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_bin_sorted_workspace(100, 4, 4, 1000, C.byref(nb)) == L.MGS_OK
    assert lib.mgs_check_capacity(None, 1000, None, None) == L.MGS_ERR_INVALID_ARG
    # pruning: n in [0, 2^31), tau in [0, 1], n = 0 enqueues nothing
    assert lib.mgs_prune_workspace(1000, C.byref(nb)) == L.MGS_OK and nb.value > 0
    assert lib.mgs_prune_workspace(-1, C.byref(nb)) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_prune_workspace(1 << 31, C.byref(nb)) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_prune_vote(None, None, 0, 0.2, 3, None, 0, None, None, None) == L.MGS_OK
    assert lib.mgs_prune_vote(None, None, 10, 1.5, 3, None, 0, None, None, None) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_prune_vote(None, None, 10, 0.2, 3, None, 0, None, None, None) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_prune_vote(None, None, 10, 0.2, 0, None, 0, None, None, None) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_prune_vote(None, None, 10, 0.2, 4, None, 0, None, None, None) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_prune_compact(None, 10, 600, None, 0, None, None, None) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_gather_planes(None, 10, 0, None, None, 10, None, 10, None) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_gather_planes(None, 10, 1, None, None, 10, None, 5, None) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_gather_planes(None, 0, 1, None, None, 10, None, 10, None) == L.MGS_ERR_INVALID_ARG
    assert lib.mgs_render_backward_workspace(100, 4, 4, 1000, 1, C.byref(nb)) == L.MGS_OK and nb.value > 0
    # invalid camera / arguments are rejected before any device work
    cam = L.mgs_camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.near_z = 0, 10, 10.0, 10.0, 0.2
    g = L.mgs_gaussians()
    g.n = 0
    proj = L.mgs_projected()
    assert lib.mgs_project(C.byref(g), C.byref(cam), None, None, 16, 1 / 255, C.byref(proj), None) \
        == L.MGS_ERR_INVALID_ARG
    assert "size" in lib.mgs_last_error().decode()
    cam.width = 10
    assert lib.mgs_project(C.byref(g), C.byref(cam), None, None, 8, 1 / 255, C.byref(proj), None) \
        == L.MGS_ERR_UNSUPPORTED
    # weight modes: the three of include/mgs.h pass the host checks (n = 0: nothing to launch),
    # anything else is rejected
    for mode in (L.MGS_WEIGHT_EQ3, L.MGS_WEIGHT_NO_DEPTH, L.MGS_WEIGHT_NO_SCALE):
        assert lib.mgs_project_weighted(C.byref(g), C.byref(cam), None, None, 16, 1 / 255, mode, C.byref(proj),
                                        None) == L.MGS_OK
    for mode in (-1, 3):
        assert lib.mgs_project_weighted(C.byref(g), C.byref(cam), None, None, 16, 1 / 255, mode, C.byref(proj),
                                        None) == L.MGS_ERR_INVALID_ARG
        assert "weight_mode" in lib.mgs_last_error().decode()
    for deg in (-1, 4):
        assert lib.mgs_enhance_project_sh(C.byref(g), deg, C.byref(cam), None, 16, 1 / 255, C.byref(proj), None,
                                          None, None) == L.MGS_ERR_INVALID_ARG
        assert "sh_degree" in lib.mgs_last_error().decode()
    assert lib.mgs_project(C.byref(g), C.byref(cam), None, None, 16, 1.5, C.byref(proj), None) \
        == L.MGS_ERR_INVALID_ARG
    # n = 0 is a valid no-op
    assert lib.mgs_project(C.byref(g), C.byref(cam), None, None, 16, 1 / 255, C.byref(proj), None) == L.MGS_OK
    assert lib.mgs_mlp_pack(None, None, None) == L.MGS_ERR_INVALID_ARG
