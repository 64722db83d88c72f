"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: tile lists bit-exact; float32 image max abs <= 1e-4 per channel
(with the ambiguity rule for pairs at the alpha cut); BF16-MLP path <= 1e-4
against the oracle's BF16 emulation, and <= 2e-2 / PSNR >= 50 dB against the
plain FP64 oracle.
"""
import math
import os
import re

import numpy as np
import pytest
import torch

import mgs_data
import oracle as O
from gpu_helpers import (compare_oit_image, oracle_project, psnr, rect_mismatches, sampled_pixel_check, say,
                         upload_projected_from_oracle)

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11531_amd as M
    M._lib.lib()
    return M


def _render_gpu(M, scene, cam, mlp=None, bg=(0, 0, 0), sorted_path=False, want_aux=False, capacity=None):
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, cam.width, cam.height, capacity=capacity)
    dm = M.DeviceMLP(mlp) if mlp is not None else None
    img = R.render(ds, cam, dm, bg=bg, sorted_path=sorted_path, want_aux=want_aux)
    torch.cuda.synchronize()
    return R, img.double().cpu()


# ------------------------------------------------------------------ projection
def test_project_matches_oracle_small(M):
    say("test_project_matches_oracle_small")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    cam = cams[0]
    R, _ = _render_gpu(M, scene, cam)
    d = R.decoded()
    pr, camt = oracle_project(scene, cam)
    vis_o = pr["visible"].numpy()
    vis_g = d["n_tiles"] > 0
    cov = pr["cov2d"].detach().numpy()
    a, b, c = cov[:, 0, 0], cov[:, 0, 1], cov[:, 1, 1]
    both = vis_o & vis_g
    assert both.sum() > 1000
    rel = lambda x, y: np.abs(x - y) / np.maximum(np.abs(y), 1e-3)
    assert rel(d["mean2d"][both], pr["mean2d"].detach().numpy()[both]).max() < 1e-5
    assert rel(d["w"][both], pr["w"].detach().numpy()[both]).max() < 1e-5
    assert np.abs(d["color"][both] - pr["color"].detach().numpy()[both]).max() < 1e-5
    assert rel(d["o_eff"][both], pr["o_eff"].detach().numpy()[both]).max() < 1e-5
    assert rel(d["depth"][both], pr["depth"].detach().numpy()[both]).max() < 1e-5
    det = a * c - b * b
    assert rel(d["A"][both], (c / det)[both]).max() < 1e-5
    assert np.abs(d["beta"][both] - (-b / c)[both]).max() < 1e-5
    assert rel(d["inv_c"][both], (1.0 / c)[both]).max() < 1e-5
    # visibility and rects agree except for splats whose support edge sits within 1e-3 px of a
    # pixel-centre boundary (the float32 extent may round to either side of it)
    diff, bad = rect_mismatches(d, pr)
    say(f"  rect / visibility differences {len(diff)}, unexplained {len(bad)}")
    assert len(bad) == 0, bad
    assert len(diff) <= 2, diff


# ------------------------------------------------------------------ lists
@pytest.mark.parametrize("W,H,n,seed", [(128, 128, 2000, 0), (200, 120, 3000, 1), (17, 33, 500, 2)])
def test_bin_lists_bit_exact_on_oracle_rects(M, W, H, n, seed):
    say(f"test_bin_lists_bit_exact_on_oracle_rects W={W} H={H} n={n}")
    scene = mgs_data.make_scene_uniform(n, seed, ls_mu=-2.5)
    cam = mgs_data.look_at((0.3, 0.1, -3.0), width=W, height=H, f=float(W))
    pr, camt = oracle_project(scene, cam)
    R = M.Renderer(n, W, H, capacity=int(pr["n_tiles"].sum()))
    upload_projected_from_oracle(R, pr, camt)
    R.bin()
    torch.cuda.synchronize()
    offs, gids = R.lists()
    o_offs, o_gids = O.bin_lists(pr["rect"], pr["n_tiles"], R.tiles_x, R.tiles_y)
    assert R.pairs() == int(pr["n_tiles"].sum())
    assert torch.equal(offs, o_offs) and torch.equal(gids, o_gids)
    # depth-sorted lists (sort key = the float32 depth held in the record)
    R.bin(sorted_path=True)
    torch.cuda.synchronize()
    offs2, gids2 = R.lists()
    depth32 = pr["depth"].detach().to(torch.float32).to(torch.float64)
    s_offs, s_gids = O.bin_lists_sorted(pr["rect"], pr["n_tiles"], depth32, R.tiles_x, R.tiles_y)
    assert torch.equal(offs2, s_offs) and torch.equal(gids2, s_gids)


@pytest.mark.parametrize("W,H,n,ls_mu", [(2048, 2048, 6000, -2.0), (1000, 700, 4000, -1.5)])
def test_bin_lists_bit_exact_large_footprints(M, W, H, n, ls_mu):
    """Gaussians covering many supertiles (up to 2^8 supertiles, tens of thousands of supertile
    entries per block of 1024 Gaussians, so the level-1 staging runs many rounds): the lists
    equal the oracle's bit for bit."""
    say(f"test_bin_lists_bit_exact_large_footprints W={W} H={H} n={n}")
    scene = mgs_data.make_scene_uniform(n, 3, ls_mu=ls_mu)
    cam = mgs_data.look_at((0.3, 0.1, -3.0), width=W, height=H, f=float(W))
    pr, camt = oracle_project(scene, cam)
    P = int(pr["n_tiles"].sum())
    R = M.Renderer(n, W, H, capacity=P)
    upload_projected_from_oracle(R, pr, camt)
    R.bin()
    torch.cuda.synchronize()
    offs, gids = R.lists()
    o_offs, o_gids = O.bin_lists(pr["rect"], pr["n_tiles"], R.tiles_x, R.tiles_y)
    say(f"  pairs {P}")
    assert R.pairs() == P
    assert torch.equal(offs, o_offs) and torch.equal(gids, o_gids)


@pytest.mark.parametrize("W,H,n,ls_mu", [(128, 128, 9000, -1.0), (200, 120, 3000, -2.5), (1000, 700, 4000, -1.5)])
def test_tile_sort_lists_equal_depth_sorted_lists(M, W, H, n, ls_mu):
    """mgs_bin + mgs_tile_sort gives the oracle's depth-sorted lists (ties by index) and exactly
    the lists of the global (tile, depth) sort; the first case has lists longer than the
    4,096 entries sorted in LDS (the chunked path)."""
    say(f"test_tile_sort_lists_equal_depth_sorted_lists W={W} H={H} n={n}")
    scene = mgs_data.make_scene_uniform(n, 5, ls_mu=ls_mu)
    cam = mgs_data.look_at((0.3, 0.1, -3.0), width=W, height=H, f=float(W))
    pr, camt = oracle_project(scene, cam)
    P = int(pr["n_tiles"].sum())
    R = M.Renderer(n, W, H, capacity=P)
    upload_projected_from_oracle(R, pr, camt)
    R.bin()
    R.tile_sort()
    torch.cuda.synchronize()
    offs, gids = R.lists()
    depth32 = pr["depth"].detach().to(torch.float32).to(torch.float64)
    s_offs, s_gids = O.bin_lists_sorted(pr["rect"], pr["n_tiles"], depth32, R.tiles_x, R.tiles_y)
    longest = int((offs[1:] - offs[:-1]).max())
    say(f"  pairs {P}, longest list {longest}")
    assert R.pairs() == P
    assert torch.equal(offs, s_offs) and torch.equal(gids, s_gids)
    R.bin(sorted_path=True)
    torch.cuda.synchronize()
    offs2, gids2 = R.lists()
    assert torch.equal(offs2, offs) and torch.equal(gids2, gids)
    if W == 128:
        assert longest > 4096


def test_tile_sort_frame_equals_global_sort_frame(M):
    """The 1M-Gaussian 1600x1063 frame (pose 0; 188 lists longer than 4,096): the two sorted
    variants give the same lists and the same image bit for bit; an overflowed binning is left
    untouched."""
    say("test_tile_sort_frame_equals_global_sort_frame")
    scene, cams, mlp, _ = mgs_data.make_config("unbounded", seed=0)
    ds, dm = M.DeviceScene(scene), M.DeviceMLP(mlp)
    cam = cams[0]
    R = M.Renderer(ds.n, cam.width, cam.height)
    a = R.render(ds, cam, dm, sorted_path=True, fused=True).clone()
    la = [t.clone() for t in R.lists()]
    b = R.render(ds, cam, dm, sorted_path="tile_sort", fused=True).clone()
    lb = R.lists()
    torch.cuda.synchronize()
    longest = int((lb[0][1:] - lb[0][:-1]).max())
    say(f"  pairs {R.pairs()}, longest list {longest}")
    assert longest > 4096
    assert torch.equal(la[0], lb[0]) and torch.equal(la[1], lb[1])
    assert torch.equal(a, b)
    # overflow: mgs_bin reports the count and builds nothing; mgs_tile_sort reads and writes nothing
    R2 = M.Renderer(ds.n, cam.width, cam.height, capacity=1024)
    R2.enhance_project(ds, M._lib.make_camera(cam), dm)
    R2.bin()
    R2.gids.fill_(7)
    R2.tile_sort()
    torch.cuda.synchronize()
    assert R2.pairs() > R2.capacity and bool((R2.gids == 7).all())


def test_bin_is_deterministic_and_overflow_is_reported(M):
    say("test_bin_is_deterministic_and_overflow_is_reported")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, 128, 128, capacity=1)
    cam_s = M._lib.make_camera(cams[0])
    R.project(ds, cam_s)
    R.bin()
    torch.cuda.synchronize()
    P = R.pairs()
    assert P > 1                       # overflow reported through n_pairs
    # ... and by the caller-side check of the C ABI, which hands back the same count
    L = M._lib
    got = L.C.c_uint64()
    assert L.lib().mgs_check_capacity(L.ptr(R.n_pairs), R.capacity, L.C.byref(got), None) == L.MGS_ERR_CAPACITY
    assert got.value == P and "exceed" in L.lib().mgs_last_error().decode()
    assert L.lib().mgs_check_capacity(L.ptr(R.n_pairs), P, None, None) == L.MGS_OK
    R.ensure_capacity(P)
    R.bin()
    assert R.check_capacity() == P
    a = [t.clone() for t in R.lists()]
    R.bin()
    b = R.lists()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ------------------------------------------------------------------ blend
def test_blend_on_oracle_records(M):
    say("test_blend_on_oracle_records")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    cam = cams[0]
    pr, camt = oracle_project(scene, cam)
    R = M.Renderer(scene["mean"].shape[1], 128, 128, capacity=int(pr["n_tiles"].sum()))
    upload_projected_from_oracle(R, pr, camt)
    R.bin()
    bg = (0.25, 0.5, 0.75)
    R.blend_oit(M._lib.make_camera(cam), bg, want_aux=True)
    torch.cuda.synchronize()
    img, aux, V, flagged = O.render_oit(pr, camt, np.array(bg), variants=True)
    err, nfail = compare_oit_image(R.image.cpu(), V, flagged, TOL)
    say(f"  max err {err:.3e}, fails {nfail}, flagged {flagged}")
    assert nfail == 0 and flagged == 0


def test_end_to_end_small_oit(M):
    say("test_end_to_end_small_oit")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    cam = cams[0]
    bg = (0.0, 0.0, 0.0)
    R, img = _render_gpu(M, scene, cam, bg=bg, want_aux=True)
    pr, camt = oracle_project(scene, cam)
    ref, aux, V, flagged = O.render_oit(pr, camt, np.array(bg), variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    say(f"  max err {err:.3e}, fails {nfail}, flagged {flagged}, P={R.pairs()}")
    assert nfail == 0 and flagged == 0
    assert float(img.std()) > 0.01
    # aux (F, D, T) follows the same sums
    a = R.aux.double().cpu()
    has = aux[3] > 0
    assert float((a[4] - aux[4]).abs().max()) < 1e-3
    assert float(((a[3] - aux[3]).abs() / aux[3].clamp(min=1e-3))[has].max()) < 1e-3


@pytest.mark.parametrize("W,H", [(96, 72), (33, 17), (1, 1), (250, 130)])
def test_end_to_end_ragged_sizes_and_background(M, W, H):
    say(f"test_end_to_end_ragged_sizes W={W} H={H}")
    scene = mgs_data.make_scene_uniform(800, 7, ls_mu=-2.8)
    cam = mgs_data.look_at((0.2, -0.4, -3.2), width=W, height=H, f=float(max(W, 8)))
    bg = (0.3, 0.6, 0.1)
    R, img = _render_gpu(M, scene, cam, bg=bg)
    pr, camt = oracle_project(scene, cam)
    ref, aux, V, flagged = O.render_oit(pr, camt, np.array(bg), variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    say(f"  max err {err:.3e}, fails {nfail}")
    assert nfail == 0


def test_empty_and_degenerate_scenes(M):
    say("test_empty_and_degenerate_scenes")
    cam = mgs_data.look_at((0, 0, -4), width=40, height=24, f=40.0)
    bg = (0.1, 0.2, 0.3)
    empty = {k: v[..., :0].copy() for k, v in mgs_data.make_scene_uniform(1, 0).items()}
    R, img = _render_gpu(M, empty, cam, bg=bg)
    assert torch.allclose(img, torch.tensor(bg, dtype=torch.float64)[:, None, None].expand(3, 24, 40))
    # all behind the camera
    sc = mgs_data.make_scene_uniform(50, 3)
    sc["mean"][2] = -10.0
    R, img = _render_gpu(M, sc, cam, bg=bg)
    assert R.pairs() == 0
    assert torch.allclose(img, torch.tensor(bg, dtype=torch.float64)[:, None, None].expand(3, 24, 40))
    # one huge Gaussian covering the whole image plus small ones
    sc = mgs_data.make_scene_uniform(30, 4)
    sc["log_scale"][:, 0] = 0.5
    sc["mean"][:, 0] = 0.0
    R, img = _render_gpu(M, sc, cam, bg=bg)
    pr, camt = oracle_project(sc, cam)
    ref, aux, V, flagged = O.render_oit(pr, camt, np.array(bg), variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    assert nfail == 0, err


@pytest.mark.parametrize("logit", [8.0, 4.1])
def test_opaque_gaussians_match_oracle(M, logit):
    """Every Gaussian in the blend's clamped loop: opacity above alpha_max (logit 8, the clamp
    binds near the centres) or just under it (logit 4.1: o = 0.9837, within the loop's margin
    of 0.99 but never clamped), against the oracle's min(a, alpha_max), over the quadrant
    patterns a mix of sizes produces."""
    say(f"test_opaque_gaussians_match_oracle[{logit}]")
    scene = mgs_data.make_scene_uniform(700, 12, ls_mu=-2.6)
    scene["opacity_logit"][:] = logit
    cam = mgs_data.look_at((0.1, 0.3, -3.0), width=120, height=88, f=110.0)
    bg = (0.2, 0.1, 0.4)
    R, img = _render_gpu(M, scene, cam, bg=bg)
    pr, camt = oracle_project(scene, cam)
    ref, aux, V, flagged = O.render_oit(pr, camt, np.array(bg), variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    say(f"  max err {err:.3e}, fails {nfail}, P={R.pairs()}")
    assert nfail == 0 and R.pairs() > 0


def test_render_is_bit_reproducible(M):
    say("test_render_is_bit_reproducible")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    _, a = _render_gpu(M, scene, cams[0])
    _, b = _render_gpu(M, scene, cams[0])
    assert torch.equal(a, b)


# ------------------------------------------------------------------ enhancement MLP
def test_enhance_matches_bf16_emulation(M):
    say("test_enhance_matches_bf16_emulation")
    scene = mgs_data.make_scene_unbounded(5000, 3)
    cam = mgs_data.circle_poses(4, 10.0, 320, 200, f=320.0)[1]
    mlp = mgs_data.make_mlp(4)
    ds = M.DeviceScene(scene)
    dm = M.DeviceMLP(mlp)
    R = M.Renderer(ds.n, cam.width, cam.height)
    R.enhance(ds, M._lib.make_camera(cam), dm)
    torch.cuda.synchronize()
    phi_g, m_g = R.phi.double().cpu(), R.omod.double().cpu()
    camt = O.camera_tensors(cam)
    p = O.scene_params(scene)
    act = O.activate(p)
    _, _, P = O.camera_space(p["mean"], camt)
    x = O.mlp_features(P, act["s"], act["q"], p["sh"])
    with torch.no_grad():
        phi_e, m_e = O.enhance(x, O.mlp_params(mlp), bf16=True)
        phi_f, m_f = O.enhance(x, O.mlp_params(mlp), bf16=False)
    e_phi = float((phi_g - phi_e).abs().max())
    e_m = float((m_g - m_e).abs().max())
    say(f"  vs bf16 emulation: phi {e_phi:.2e} m {e_m:.2e}; vs fp64: phi "
        f"{float((phi_g - phi_f).abs().max()):.2e} m {float((m_g - m_f).abs().max()):.2e}")
    assert e_phi < 2e-2 * float(phi_e.abs().max()) and e_m < 1e-2
    # the bulk agrees much more tightly (rare bf16 rounding flips aside)
    assert float((phi_g - phi_e).abs().median()) < 1e-5 and float((m_g - m_e).abs().median()) < 1e-5
    assert float((phi_g - phi_f).abs().max()) < 5e-2 and float((m_g - m_f).abs().max()) < 2e-2


def test_end_to_end_with_mlp(M):
    say("test_end_to_end_with_mlp")
    scene = mgs_data.make_scene_unbounded(20000, 5)
    cam = mgs_data.circle_poses(8, 10.0, 200, 132, f=200.0)[3]
    mlp = mgs_data.make_mlp(6)
    bg = (0.0, 0.0, 0.0)
    R, img = _render_gpu(M, scene, cam, mlp=mlp, bg=bg)
    pr_e, camt = oracle_project(scene, cam, mlp=mlp, bf16=True)
    ref_e, _, V, flagged = O.render_oit(pr_e, camt, np.array(bg), mode="binned", variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    pr_f, _ = oracle_project(scene, cam, mlp=mlp, bf16=False)
    ref_f, _ = O.render_oit(pr_f, camt, np.array(bg), mode="binned")
    e64 = float((img - ref_f).abs().max())
    ps = psnr(img, ref_f)
    say(f"  vs bf16-emulation: max {err:.3e} fails {nfail}; vs fp64: max {e64:.3e} psnr {ps:.1f} dB")
    assert e64 <= 2e-2 and ps >= 50.0
    # pixels off by more than 1e-4 from the emulation come only from bf16 rounding flips
    assert nfail <= max(2, img[0].numel() // 2000)


@pytest.mark.parametrize("weight_mode", [1, 2])
def test_weight_ablations_match_oracle(M, weight_mode):
    """Eq. 3 without depth / without scale (Table 3 ablations): weights and image against the
    oracle's BF16 emulation, and the fused and unfused projections agree bit for bit."""
    say(f"test_weight_ablations_match_oracle[{weight_mode}]")
    scene = mgs_data.make_scene_unbounded(20000, 5)
    cam = mgs_data.circle_poses(8, 10.0, 200, 132, f=200.0)[3]
    mlp = mgs_data.make_mlp(6)
    ds, dm = M.DeviceScene(scene), M.DeviceMLP(mlp)
    R = M.Renderer(ds.n, cam.width, cam.height)
    img = R.render(ds, cam, dm, fused=True, weight_mode=weight_mode).double().cpu()
    d = R.decoded()
    R2 = M.Renderer(ds.n, cam.width, cam.height)
    img2 = R2.render(ds, cam, dm, fused=False, weight_mode=weight_mode).double().cpu()
    torch.cuda.synchronize()
    assert torch.equal(img, img2) and torch.equal(R.splat, R2.splat)
    pr, camt = oracle_project(scene, cam, mlp=mlp, bf16=True, weight_mode=weight_mode)
    both = pr["visible"].numpy() & (d["n_tiles"] > 0)
    assert both.sum() > 1000
    w_o = pr["w"].detach().numpy()[both]
    # w carries phi, whose float32 MLP differs from the emulation by rare bf16 rounding flips
    # (as in test_enhance_matches_bf16_emulation): a loose bound on the worst Gaussian, a tight
    # one on the median
    rel = np.abs(d["w"][both] - w_o) / np.maximum(np.abs(w_o), 1.0)
    pr0, _ = oracle_project(scene, cam, mlp=mlp, bf16=True)
    assert not np.allclose(pr0["w"].detach().numpy()[both], w_o)      # the mode changed the weights
    _, _, V, flagged = O.render_oit(pr, camt, np.array((0.0, 0.0, 0.0)), mode="binned", variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    say(f"  w max rel {rel.max():.2e} median {np.median(rel):.2e}; image max {err:.3e} fails {nfail}")
    assert rel.max() < 2e-2 and np.median(rel) < 1e-5
    assert nfail <= max(2, img[0].numel() // 2000)


# ------------------------------------------------------------------ sorted comparison path
def test_sorted_path_matches_oracle(M):
    say("test_sorted_path_matches_oracle")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    cam = cams[0]
    bg = (0.2, 0.1, 0.4)
    R, img = _render_gpu(M, scene, cam, bg=bg, sorted_path=True)
    pr, camt = oracle_project(scene, cam)
    ref, flags = O.render_sorted(pr, camt, np.array(bg), return_flags=True)
    err = (img - ref).abs().amax(dim=0)
    ok = ~flags
    say(f"  max err (unflagged) {float(err[ok].max()):.3e}, flagged {int(flags.sum())}")
    assert float(err[ok].max()) <= TOL
    assert int(flags.sum()) <= img[0].numel() // 100


# ------------------------------------------------------------------ full-size workload
@pytest.mark.parametrize("sorted_path", [False, True])
def test_unbounded_full_size_sampled(M, sorted_path):
    """1M Gaussians at 1600x1063 (the benchmark workload): lists bit-exact on oracle rects,
    image checked at sampled pixels against the oracle's per-pixel evaluation."""
    say(f"test_unbounded_full_size_sampled sorted={sorted_path}")
    scene, cams, mlp, _ = mgs_data.make_config("unbounded", seed=0)
    cam = cams[0]
    bg = (0.0, 0.0, 0.0)
    R, img = _render_gpu(M, scene, cam, mlp=mlp, bg=bg, sorted_path=sorted_path)
    say(f"  P = {R.pairs()}")
    pr, camt = oracle_project(scene, cam, mlp=mlp, bf16=True)
    lists = O.bin_lists(pr["rect"], pr["n_tiles"], R.tiles_x, R.tiles_y)
    if sorted_path:
        return _sorted_sampled(img, pr, camt, bg, lists)
    worst, fails = sampled_pixel_check(img, pr, camt, bg, lists, 1500, 11, TOL)
    say(f"  sampled: worst {worst:.3e} fails {fails}")
    assert fails <= 3          # bf16 rounding flips of phi / m (see test_end_to_end_with_mlp)
    # lists: the GPU binning of the oracle's own rects is bit-exact
    upload_projected_from_oracle(R, pr, camt)
    R.ensure_capacity(int(pr["n_tiles"].sum()) + 16)
    R.bin()
    torch.cuda.synchronize()
    offs, gids = R.lists()
    assert torch.equal(offs, lists[0]) and torch.equal(gids, lists[1])


def _sorted_sampled(img, pr, camt, bg, lists):
    rng = np.random.default_rng(5)
    H, W = camt["H"], camt["W"]
    tiles_x = (W + 15) // 16
    offs, gids = lists
    bad = 0
    for p in rng.choice(H * W, 600, replace=False):
        j, i = divmod(int(p), W)
        t = (j // 16) * tiles_x + i // 16
        g = gids[int(offs[t]):int(offs[t + 1])]
        if g.numel() == 0:
            continue
        sub = {k: (v[g] if torch.is_tensor(v) and v.dim() > 0 and v.shape[0] == pr["depth"].shape[0] else v)
               for k, v in pr.items()}
        sub_img, flags = _render_pixel_sorted(sub, i, j, bg)
        if flags:
            continue
        bad += float((img[:, j, i] - sub_img).abs().max()) > TOL
    assert bad <= 3


def _render_pixel_sorted(sub, i, j, bg):
    dep = sub["depth"].detach()
    order = torch.sort(dep, stable=True).indices
    m2, con, o, col = sub["mean2d"][order], sub["conic"][order], sub["o_eff"][order], sub["color"][order]
    dx = i + 0.5 - m2[:, 0]
    dy = j + 0.5 - m2[:, 1]
    a = o * torch.exp(-0.5 * (con[:, 0] * dx * dx + 2 * con[:, 1] * dx * dy + con[:, 2] * dy * dy))
    T = 1.0
    C = torch.zeros(3, dtype=torch.float64)
    flag = False
    for k in range(a.numel()):
        ak = float(a[k])
        if abs(math.log(max(ak, 1e-300) / O.ALPHA_MIN)) < O.AMBIG_LOG:
            flag = True
        if ak < O.ALPHA_MIN:
            continue
        if T < O.T_STOP:
            break
        if abs(T / O.T_STOP - 1) < 1e-3:
            flag = True
        al = min(ak, O.ALPHA_MAX)
        C += al * T * col[k]
        T *= 1 - al
    return C + T * torch.tensor(np.asarray(bg, np.float64)), flag


def test_fused_enhance_project_equals_separate_calls(M):
    say("test_fused_enhance_project_equals_separate_calls")
    scene = mgs_data.make_scene_unbounded(30001, 8)
    cam = mgs_data.circle_poses(8, 10.0, 240, 160, f=240.0)[5]
    mlp = mgs_data.make_mlp(9)
    ds = M.DeviceScene(scene)
    dm = M.DeviceMLP(mlp)
    a = M.Renderer(ds.n, cam.width, cam.height)
    b = M.Renderer(ds.n, cam.width, cam.height)
    ia = a.render(ds, cam, dm, fused=False).clone()
    ib = b.render(ds, cam, dm, fused=True).clone()
    torch.cuda.synchronize()
    assert torch.equal(a.splat, b.splat) and torch.equal(a.n_tiles, b.n_tiles)
    assert torch.equal(a.phi, b.phi) and torch.equal(a.omod, b.omod)
    assert torch.equal(ia, ib)


def _split_range():
    """Gaussians per range of the split blend (SPLIT_RANGE of the kernels' index_math.h)."""
    text = open(os.path.join(os.path.dirname(__file__), "..", "paper_2603_11531_amd", "csrc", "index_math.h")).read()
    return int(re.search(r"constexpr uint32_t SPLIT_RANGE = (\d+);", text).group(1))


def test_split_tile_longer_than_255_full_ranges(M):
    """One tile with more than 255 x SPLIT_RANGE Gaussians: its list is cut into 255 ranges of
    ceil(L / 255) > SPLIT_RANGE (the long-list rule of the split plan), merged in order."""
    say("test_split_tile_longer_than_255_full_ranges")
    rl = _split_range()
    scene = mgs_data.make_scene_uniform(int(255 * rl * 1.04), 21, half=0.5, ls_mu=-4.5)
    cam = mgs_data.look_at((0.0, 0.0, -4.0), width=16, height=16, f=16.0)
    bg = (0.1, 0.2, 0.3)
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, cam.width, cam.height, capacity=ds.n)
    split_img = R.render(ds, cam, bg=bg, split=True).double().cpu()
    offs, _ = R.lists()
    L = int(offs[1] - offs[0])
    say(f"  one tile, list length {L}")
    assert L > 255 * rl
    tile_img = R.render(ds, cam, bg=bg, split=False).double().cpu()
    # L-term float32 sums in two different orders (255 ranges vs four waves)
    d = float((split_img - tile_img).abs().max())
    say(f"  split vs per-tile blend: {d:.3e}")
    assert d < TOL
    pr, camt = oracle_project(scene, cam)
    ref, aux, V, flagged = O.render_oit(pr, camt, np.array(bg), mode="binned", variants=True)
    err, nfail = compare_oit_image(split_img, V, flagged, TOL)
    say(f"  split vs oracle: max {err:.3e} fails {nfail} flagged {flagged}")
    assert nfail == 0


def test_split_tile_blend_matches_oracle_and_per_tile_blend(M):
    """Dense tiles (lists several SPLIT_RANGE-Gaussian ranges long) through the split blend."""
    say("test_split_tile_blend_matches_oracle_and_per_tile_blend")
    scene = mgs_data.make_scene_uniform(40000 * _split_range() // 1024, 12, ls_mu=-3.0)
    cam = mgs_data.look_at((0.1, -0.2, -4.0), width=136, height=120, f=136.0)
    bg = (0.2, 0.3, 0.4)
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, cam.width, cam.height)
    split_img = R.render(ds, cam, bg=bg, split=True, want_aux=True).double().cpu()
    offs, _ = R.lists()
    longest = int((offs[1:] - offs[:-1]).max())
    say(f"  P={R.pairs()} longest list {longest}")
    assert longest > 3 * _split_range()
    tile_img = R.render(ds, cam, bg=bg, split=False).double().cpu()
    assert float((split_img - tile_img).abs().max()) < 2e-6
    pr, camt = oracle_project(scene, cam)
    ref, aux, V, flagged = O.render_oit(pr, camt, np.array(bg), mode="binned", variants=True)
    err, nfail = compare_oit_image(split_img, V, flagged, TOL)
    say(f"  split vs oracle: max {err:.3e} fails {nfail} flagged {flagged}")
    assert nfail == 0


@pytest.mark.parametrize("W,H", [(2048, 1024), (2049, 1023), (1600, 1312), (2560, 1440), (3840, 2160), (4160, 4112)])
def test_split_blend_views_over_one_plan_chunk(M, W, H):
    """Views around and above 8,192 tiles (one chunk of the split plan): exactly one chunk
    (2048x1024), a second chunk of 64 tiles with ragged edges (2049x1023) or of 8 tiles
    (1600x1312), two and four chunks (the longest-first plan over several chunks), nine (the
    tile-order multi-pass plan).  Dense middle tiles are split; the image equals the per-tile
    blend's and the oracle's at sampled pixels."""
    say(f"test_split_blend_views_over_one_plan_chunk W={W} H={H}")
    scene = mgs_data.make_scene_uniform(100000, 31, ls_mu=-3.1)
    cam = mgs_data.look_at((0.1, 0.2, -4.0), width=W, height=H, f=float(W) * 0.6)
    bg = (0.25, 0.1, 0.4)
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, W, H)
    split_img = R.render(ds, cam, bg=bg, split=True).double().cpu()
    offs, gids = R.lists()
    n = offs[1:] - offs[:-1]
    chunks = -(-R.tiles_x * R.tiles_y // 8192)
    say(f"  tiles {R.tiles_x * R.tiles_y} ({chunks} plan chunks), P={R.pairs()}, longest {int(n.max())}, "
        f"split tiles {int((n > _split_range()).sum())}, empty {int((n == 0).sum())}")
    assert int((n > _split_range()).sum()) > 0 and int((n == 0).sum()) > 0
    tile_img = R.render(ds, cam, bg=bg, split=False).double().cpu()
    d = float((split_img - tile_img).abs().max())
    say(f"  split vs per-tile blend: {d:.3e}")
    assert d < 2e-6
    pr, camt = oracle_project(scene, cam)
    lists = O.bin_lists(pr["rect"], pr["n_tiles"], R.tiles_x, R.tiles_y)
    worst, fails = sampled_pixel_check(split_img, pr, camt, bg, lists, 400, 13, TOL)
    say(f"  sampled vs oracle: worst {worst:.3e} fails {fails}")
    assert fails == 0


def test_blend_census_counts_match_oracle(M):
    """mgs_blend_census: list entries equal the oracle's pair count; contributing pixel-Gaussian
    pairs equal the oracle's count of alpha >= alpha_min pairs up to pairs in the ambiguity band;
    the executed evaluations lie between the contributing pairs and 256 P."""
    say("test_blend_census_counts_match_oracle")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    cam = cams[0]
    R, _ = _render_gpu(M, scene, cam)
    P, executed, contributing = R.census(M._lib.make_camera(cam))
    pr, camt = oracle_project(scene, cam)
    offs, gids = O.bin_lists(pr["rect"], pr["n_tiles"], pr["tiles_x"], pr["tiles_y"])
    pix = O.pixel_grid(camt["W"], camt["H"])
    ref, amb = 0, 0
    with torch.no_grad():
        for t in range(pr["tiles_x"] * pr["tiles_y"]):
            g = gids[offs[t]:offs[t + 1]]
            if g.numel() == 0:
                continue
            tx, ty = t % pr["tiles_x"], t // pr["tiles_x"]
            ii = torch.arange(tx * 16, min(camt["W"], tx * 16 + 16))
            jj = torch.arange(ty * 16, min(camt["H"], ty * 16 + 16))
            pp = pix[(jj[:, None] * camt["W"] + ii[None, :]).reshape(-1)]
            _, _, _, cnt, _, n_amb = O.eval_pixels_oit(pp, pr, g, track_ambiguous=True)
            ref += int(cnt.sum())
            amb += int(n_amb.sum())
    say(f"  P {P}, executed {executed} ({executed / (256 * P):.3f} of 256 P), contributing {contributing} "
        f"(oracle {ref}, ambiguous {amb})")
    assert P == int(offs[-1]) == R.pairs()
    assert abs(contributing - ref) <= amb
    assert contributing <= executed <= 256 * P and executed % 64 == 0
