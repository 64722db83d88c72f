"""Whole frames at the benchmark sizes through the C ABI against the FP64 oracle.

1,000,000 Gaussians at 1600x1063 (the unbounded workload, pose 0) and 3,000,000 at
1920x1080 (the large workload, pose 0), every pixel compared, no sampling:

* float32 path (enhancement MLP off, the oracle's answer is unique up to the ambiguous
  alpha cut): max abs <= 1e-4 per channel against one admissible oracle image, every pixel;
* BF16-MLP path in the launch sequence the benchmark times (fused enhance + project, split
  blend): max abs <= 2e-2 and PSNR >= 50 dB against the plain FP64 oracle, and the count of
  pixels off the oracle's BF16 emulation by more than 1e-4 (bf16 rounding flips of phi / m);
* sorted comparison path: every pixel the oracle does not flag (depth ties below the float32
  key's resolution, transmittance at the stop value, ambiguous alpha) within 1e-4.

The oracle evaluates each tile's pixels over the tile's list (binned mode, pinned equal to
brute force on small scenes).
"""
import numpy as np
import pytest
import torch

import mgs_data
import oracle as O
from gpu_helpers import compare_oit_image, oracle_project, psnr, rect_mismatches, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

TOL = 1e-4
_CACHE = {}


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11531_amd as M
    M._lib.lib()
    return M


def _workload(name):
    if name not in _CACHE:
        scene, cams, mlp, _ = mgs_data.make_config(name, seed=0)
        _CACHE.clear()
        _CACHE[name] = (scene, cams[0], mlp)
    return _CACHE[name]


def _gpu(M, scene, cam, mlp=None, sorted_path=False, bg=(0.0, 0.0, 0.0)):
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, cam.width, cam.height)
    dm = M.DeviceMLP(mlp) if mlp is not None else None
    img = R.render(ds, cam, dm, bg=bg, sorted_path=sorted_path, fused=mlp is not None).double().cpu()
    torch.cuda.synchronize()
    return R, img


@pytest.mark.parametrize("name", ["unbounded", "large"])
def test_full_frame_float32_every_pixel(M, name):
    say(f"test_full_frame_float32_every_pixel[{name}]")
    scene, cam, _ = _workload(name)
    bg = (0.0, 0.0, 0.0)
    R, img = _gpu(M, scene, cam)
    say(f"  {cam.width}x{cam.height}, P = {R.pairs()}")
    pr, camt = oracle_project(scene, cam)
    lists = O.bin_lists(pr["rect"], pr["n_tiles"], pr["tiles_x"], pr["tiles_y"])
    # pair counts agree up to rects whose support edge float32 may put on either side of a
    # pixel-centre boundary (those pairs are at alpha_min: the ambiguity rule covers them)
    diff, bad = rect_mismatches(R.decoded(), pr)
    say(f"  pairs GPU {R.pairs()} oracle {int(pr['n_tiles'].sum())}; rect differences {len(diff)}, "
        f"unexplained {len(bad)}")
    assert len(bad) == 0, bad[:10]
    assert abs(R.pairs() - int(pr["n_tiles"].sum())) <= 4 * len(diff)
    with torch.no_grad():
        _, _, V, flagged = O.render_oit(pr, camt, np.array(bg), mode="binned", lists=lists, variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    say(f"  max err {err:.3e}, pixels over 1e-4: {nfail}, pixels with > 2 ambiguous pairs: {flagged}")
    # a pixel with more than two ambiguous pairs has admissible images the oracle does not list
    assert nfail <= flagged and flagged <= img[0].numel() // 2000
    assert float(img.std()) > 1e-3            # the frame is not trivially uniform


@pytest.mark.parametrize("name", ["unbounded", "large"])
def test_full_frame_bf16_mlp_bench_launch(M, name):
    say(f"test_full_frame_bf16_mlp_bench_launch[{name}]")
    scene, cam, mlp = _workload(name)
    bg = (0.0, 0.0, 0.0)
    R, img = _gpu(M, scene, cam, mlp=mlp)
    with torch.no_grad():
        pr64, camt = oracle_project(scene, cam, mlp=mlp, bf16=False)
        ref64, _ = O.render_oit(pr64, camt, np.array(bg), mode="binned")
    e64, ps = float((img - ref64).abs().max()), psnr(img, ref64)
    say(f"  vs FP64: max {e64:.3e}, PSNR {ps:.1f} dB")
    assert e64 <= 2e-2 and ps >= 50.0
    if name != "unbounded":
        return
    with torch.no_grad():
        pre, _ = oracle_project(scene, cam, mlp=mlp, bf16=True)
        _, _, V, flagged = O.render_oit(pre, camt, np.array(bg), mode="binned", variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    # phi / m: the float32 MLP differs from the emulation only where a bf16 rounding flips
    dphi = (R.phi.double().cpu() - pre["phi"]).abs()
    dm = (R.omod.double().cpu() - pre["m"]).abs()
    flipped = float(((dphi > 1e-5 * (1 + pre["phi"].abs())) | (dm > 1e-6)).double().mean())
    say(f"  vs BF16 emulation: max {err:.3e}, pixels over 1e-4: {nfail} of {img[0].numel()}; "
        f"Gaussians with a flipped rounding: {flipped:.2%}")
    assert flipped < 0.01
    assert nfail <= img[0].numel() // 2000


@pytest.mark.parametrize("name", ["unbounded", "large"])
def test_full_frame_sorted_unflagged_pixels(M, name):
    say(f"test_full_frame_sorted_unflagged_pixels[{name}]")
    scene, cam, _ = _workload(name)
    bg = (0.0, 0.0, 0.0)
    R, img = _gpu(M, scene, cam, sorted_path=True)
    pr, camt = oracle_project(scene, cam)
    with torch.no_grad():
        ref, flags = O.render_sorted(pr, camt, np.array(bg), mode="binned", return_flags=True)
    err = (img - ref).abs().amax(dim=0)
    ok = ~flags
    worst = float(err[ok].max())
    say(f"  unflagged max err {worst:.3e}; flagged {int(flags.sum())} of {flags.numel()}; "
        f"flagged max err {float(err[flags].max()) if bool(flags.any()) else 0.0:.3e}")
    assert worst <= TOL
    # the flagged share is what a float32 key and transmittance cannot decide (8.5% at 1M
    # Gaussians, 13% at 3M); the bound only guards against a flag rule that hides the frame
    assert int(flags.sum()) <= flags.numel() // 5
