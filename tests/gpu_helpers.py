"""Shared helpers of the GPU parity tests (imported by tests only).

The HIP side is reached only through the C ABI (paper_2603_11531_amd); the
expected values come only from the FP64 oracle on the same seeded inputs.
"""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

import oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_project(scene, cam, mlp=None, bf16=False, tile=16, weight_mode=O.WEIGHT_EQ3):
    camt = O.camera_tensors(cam)
    p = O.scene_params(scene)
    phi = m = None
    if mlp is not None:
        act = O.activate(p)
        _, _, P = O.camera_space(p["mean"], camt)
        phi, m = O.enhance(O.mlp_features(P, act["s"], act["q"], p["sh"]), O.mlp_params(mlp), bf16=bf16)
    with torch.no_grad():
        return O.project(p, camt, phi, m, tile, weight_mode), camt


def compare_oit_image(gpu_img, variants, flagged, tol):
    """Per pixel, the GPU result must be within tol (max over channels) of one admissible
    oracle result.  Returns (max error over pixels, number of pixels failing)."""
    g = torch.as_tensor(gpu_img, dtype=torch.float64)
    err = (variants - g[None]).abs().amax(dim=1)          # (4, H, W)
    best = err.min(dim=0).values
    return float(best.max()), int((best > tol).sum())


def psnr(a, b):
    mse = float(((torch.as_tensor(a, dtype=torch.float64) - torch.as_tensor(b, dtype=torch.float64)) ** 2).mean())
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def sampled_pixel_check(gpu_img, proj, camt, bg, lists, n_samples, seed, tol):
    """Evaluate the oracle at sampled pixels (each over its tile's list) and compare."""
    H, W = camt["H"], camt["W"]
    rng = np.random.default_rng(seed)
    pix_idx = rng.choice(H * W, size=min(n_samples, H * W), replace=False)
    offs, gids = lists
    tiles_x = (W + 15) // 16
    bgt = torch.tensor(np.asarray(bg, np.float64))
    worst, fails = 0.0, 0
    img = torch.as_tensor(gpu_img, dtype=torch.float64)
    for p in pix_idx:
        j, i = divmod(int(p), W)
        t = (j // 16) * tiles_x + (i // 16)
        g = gids[int(offs[t]):int(offs[t + 1])]
        pix = torch.tensor([[i + 0.5, j + 0.5]], dtype=torch.float64)
        if g.numel() == 0:
            V = bgt[None, None, :].expand(4, 1, 3)
        else:
            N, D, T, _, amb, _ = O.eval_pixels_oit(pix, proj, g, track_ambiguous=True)
            V = O.oit_pixel_variants(N, D, T, amb, bgt)
        e = float((V[:, 0, :] - img[:, j, i][None]).abs().amax(dim=1).min())
        worst = max(worst, e)
        fails += e > tol
    return worst, fails


def upload_projected_from_oracle(R, proj, camt):
    """Write the oracle's projected Gaussians into the GPU record (test harness only).

    Used to test mgs_bin / mgs_blend_* in isolation on oracle inputs; the record
    encoding is the documented mgs_projected layout.
    """
    LOG2E = 1.4426950408889634
    cov = proj["cov2d"].detach()
    a, b, c = cov[:, 0, 0], cov[:, 0, 1], cov[:, 1, 1]
    det = a * c - b * b
    o = proj["o_eff"].detach()
    rec = torch.stack([
        proj["mean2d"][:, 0].detach(), proj["mean2d"][:, 1].detach(), torch.log2(o.clamp(min=1e-30)),
        proj["w"].detach(),
        -0.5 * LOG2E * c / det, -b / c, -0.5 * LOG2E / c, proj["depth"].detach(),
        proj["color"][:, 0].detach(), proj["color"][:, 1].detach(), proj["color"][:, 2].detach(), o], dim=1)
    R.splat.copy_(rec.to(torch.float32).to(R.device))
    rect = proj["rect"]
    packed = torch.stack([rect[:, 0] | (rect[:, 1] << 16), rect[:, 2] | (rect[:, 3] << 16)], 1)
    R.rect.copy_(packed.to(torch.int32).to(R.device))
    R.n_tiles.copy_(proj["n_tiles"].to(torch.int32).to(R.device))
