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


def oracle_project(scene, cam, mlp=None, bf16=False, tile=16, weight_mode=O.WEIGHT_EQ3, sortfree=None):
    """The oracle's projection of a scene; ``sortfree`` = (sigma, beta) selects Eq. 1's weight."""
    camt = O.camera_tensors(cam)
    p = O.scene_params(scene)
    phi = m = None
    with torch.no_grad():
        if mlp is not None:
            act = O.activate(p)
            _, _, P = O.camera_space(p["mean"], camt)
            phi, m = O.enhance(O.mlp_features(P, act["s"], act["q"], p["sh"]), O.mlp_params(mlp), bf16=bf16)
        if sortfree is not None:
            weight_mode = O.WEIGHT_SORTFREE
            sortfree = tuple(O.to64(np.asarray(v)) for v in sortfree)
        return O.project(p, camt, phi, m, tile, weight_mode, sortfree), camt


def rect_mismatches(decoded, pr, tol_px=1e-3):
    """Gaussians whose GPU tile rect or visibility differs from the oracle's, and the subset of
    them NOT explained by an edge case float32 may decide either way: a support edge
    m +- e - 1/2 within tol_px plus the Gaussian's screen-position error bound of a pixel-centre
    boundary, an effective opacity within the ambiguity band of alpha_min, or a depth at the near
    plane.  Returns (differing indices, unexplained indices)."""
    vis_o = pr["visible"].numpy()
    vis_g = np.asarray(decoded["n_tiles"]) > 0
    both = vis_o & vis_g
    diff = np.nonzero((vis_o != vis_g) | (np.any(np.asarray(decoded["rect"]) != pr["rect"].numpy(), axis=1) & both))[0]
    cov = pr["cov2d"].detach().numpy()
    o = pr["o_eff"].detach().numpy()
    m2 = pr["mean2d"].detach().numpy()
    pos = pr["pos_err"].numpy()
    dep = pr["depth"].detach().numpy()
    bad = []
    for g in diff:
        k = 2.0 * np.log(max(o[g], O.ALPHA_MIN) / O.ALPHA_MIN)
        ex, ey = np.sqrt(k * cov[g, 0, 0]), np.sqrt(k * cov[g, 1, 1])
        edges = np.array([m2[g, 0] - ex - 0.5, m2[g, 0] + ex - 0.5, m2[g, 1] - ey - 0.5, m2[g, 1] + ey - 0.5])
        gap = float(np.abs(edges - np.round(edges)).min())
        opacity_at_cut = abs(np.log(max(o[g], 1e-300) / O.ALPHA_MIN)) < O.AMBIG_LOG
        near_plane = abs(dep[g] - 0.2) < 1e-6
        if not (gap < tol_px + pos[g] or opacity_at_cut or near_plane):
            bad.append(int(g))
    return diff, np.asarray(bad, np.int64)


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
