"""The no-allocation split blend (mgs_blend_oit_split_noalloc, workspace in a static device
array) against mgs_blend_oit_split with a caller workspace: two calls in a row, the second on
a smaller input, bit-identical images and aux (the same kernels run on the same lists); and a
view whose workspace exceeds the array is refused before any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

import mgs_data
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11531_amd as M
    M._lib.lib()
    return M


def _noalloc(M, R, cam_s, bg, out, aux):
    L = M._lib
    return L.lib().mgs_blend_oit_split_noalloc(C.byref(R.proj), L.ptr(R.tile_offsets), L.ptr(R.gids),
                                               L.ptr(R.n_pairs), R.capacity, C.byref(cam_s), L.MGS_TILE,
                                               L.bg_array(bg), M.render.ALPHA_MIN, M.render.ALPHA_MAX, L.ptr(out),
                                               L.ptr(aux), L.stream_ptr())


def test_noalloc_split_blend_equals_workspace_call(M):
    L = M._lib
    cases = [  # a view of two split-plan chunks (14,400 tiles; the chunk totals in the scratch too),
        # then dense lists (split tiles, partial sums in the scratch), then a smaller view
        (mgs_data.make_scene_uniform(30000, 31, ls_mu=-3.1), (0.1, 0.2, -4.0), 2560, 1440, (0.25, 0.1, 0.4), 0.6),
        (mgs_data.make_scene_uniform(40000, 12, ls_mu=-3.0), (0.1, -0.2, -4.0), 136, 120, (0.2, 0.3, 0.4), 1.0),
        (mgs_data.make_scene_uniform(3000, 5, ls_mu=-2.8), (0.3, 0.1, -3.5), 72, 40, (0.5, 0.1, 0.0), 1.0),
    ]
    for k, (scene, eye, W, H, bg, fs) in enumerate(cases):
        say(f"test_noalloc_split_blend_equals_workspace_call: call {k + 1}, {scene['mean'].shape[1]} Gaussians "
            f"{W}x{H}")
        cam = mgs_data.look_at(eye, width=W, height=H, f=float(W) * fs)
        ds = M.DeviceScene(scene)
        R = M.Renderer(ds.n, W, H)
        ref = R.render(ds, cam, bg=bg, split=True, want_aux=True).clone()
        ref_aux = R.aux.clone()
        offs, _ = R.lists()
        longest = int((offs[1:] - offs[:-1]).max())
        out = torch.full_like(ref, -1.0)
        aux = torch.full_like(ref_aux, -1.0)
        L.check(_noalloc(M, R, L.make_camera(cam), bg, out, aux))
        torch.cuda.synchronize()
        say(f"  P = {R.pairs()}, longest list {longest}")
        if k == 0:
            assert R.tiles_x * R.tiles_y > 8192
        if k == 1:
            assert longest > 3 * 1024
        assert torch.equal(out, ref) and torch.equal(aux, ref_aux)


def test_noalloc_refuses_a_workspace_beyond_the_scratch(M):
    say("test_noalloc_refuses_a_workspace_beyond_the_scratch")
    L = M._lib
    R = M.Renderer(100, 1920, 1080, capacity=1024)
    cam_s = L.make_camera(mgs_data.look_at((0, 0, -4), width=1920, height=1080, f=1920.0))
    nb = C.c_size_t()
    big_cap = 200_000_000
    L.check(L.lib().mgs_blend_oit_split_workspace(R.tiles_x, R.tiles_y, big_cap, C.byref(nb)))
    assert nb.value > L.MGS_NOALLOC_SCRATCH_BYTES
    rc = L.lib().mgs_blend_oit_split_noalloc(C.byref(R.proj), L.ptr(R.tile_offsets), L.ptr(R.gids),
                                             L.ptr(R.n_pairs), big_cap, C.byref(cam_s), L.MGS_TILE,
                                             L.bg_array((0, 0, 0)), 1 / 255, 0.99, L.ptr(R.image), None,
                                             L.stream_ptr())
    assert rc == L.MGS_ERR_CAPACITY
    assert b"no-allocation scratch" in L.lib().mgs_last_error()
    torch.cuda.synchronize()
