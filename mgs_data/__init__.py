"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module only draws random numbers and lays them out; it holds none of the
renderer's arithmetic (no projection, no colour, no weighting, no blending).
Everything it returns is plain numpy float32/int arrays:

* scene: ``mean [3][N]``, ``log_scale [3][N]``, ``quat [4][N]`` (w, x, y, z,
  unnormalised), ``opacity_logit [N]``, ``sh [12][N]`` (plane 3k+ch: SH
  coefficient k in 0..3, colour channel ch in r, g, b).  These are the
  per-Gaussian attributes of the paper's 3D Gaussian representation
  (Appendix B) restricted to first-order SH (Sec. 3.2).
* camera: world->camera rotation ``R`` (row-major 3x3), translation ``t``,
  focal lengths, principal point, image size and near plane.
* mlp: FP32 master weights of the view-dependent enhancement MLP (Eq. 4):
  22 -> 64 -> 64 -> {phi, opacity} heads.

Distributions follow the workload recipes of the generators below (synthetic
stand-ins for the paper's Mip-NeRF 360 / Tanks&Temples / Deep Blending scenes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Camera", "look_at", "make_scene_uniform", "make_scene_unbounded",
    "make_scene_ball", "make_mlp", "circle_poses", "spline_poses",
    "make_config", "tiny_scene", "perturb_scene", "MLP_IN", "MLP_HIDDEN", "make_mlp_f", "MLP_F_WIDTHS", "with_sh_degree",
    "make_nvq", "NVQ_GROUPS", "NVQ_DIM", "NVQ_CODEWORDS",
]

MLP_IN = 22       # [P(3), s(3), q(4), Y(12)]
MLP_HIDDEN = 64   # two hidden layers of width 64 (the benchmark MLP shape)


@dataclass
class Camera:
    R: np.ndarray            # (3, 3) float32, world -> camera rows (right, down, forward)
    t: np.ndarray            # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2

    def as_dict(self):
        return dict(R=self.R, t=self.t, fx=self.fx, fy=self.fy, cx=self.cx,
                    cy=self.cy, width=self.width, height=self.height, near=self.near)


def look_at(eye, target=(0.0, 0.0, 0.0), width=128, height=128, f=None, near=0.2):
    """Pinhole camera at ``eye`` looking at ``target``; world up is -y.

    Camera axes: x right, y down, z forward (the camera looks along +z).
    """
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    down_w = np.array([0.0, 1.0, 0.0])
    right = np.cross(down_w, fwd)
    if np.linalg.norm(right) < 1e-9:          # looking straight up/down
        right = np.array([1.0, 0.0, 0.0])
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)
    t = (-R.astype(np.float64) @ eye).astype(np.float32)
    f = float(width if f is None else f)
    return Camera(R=R, t=t, fx=f, fy=f, cx=width / 2.0, cy=height / 2.0,
                  width=int(width), height=int(height), near=near)


def _random_quats(rng, n):
    return rng.normal(0.0, 1.0, size=(n, 4))


def _soa(mean, log_scale, quat, opac, sh):
    n = mean.shape[0]
    return dict(
        mean=np.ascontiguousarray(mean.T, dtype=np.float32),
        log_scale=np.ascontiguousarray(log_scale.T, dtype=np.float32),
        quat=np.ascontiguousarray(quat.T, dtype=np.float32),
        opacity_logit=np.ascontiguousarray(opac, dtype=np.float32),
        sh=np.ascontiguousarray(sh.reshape(n, 12).T, dtype=np.float32),
    )


def make_scene_uniform(n, seed, half=1.0, ls_mu=-3.5, ls_sd=0.5, op_sd=1.5, sh_sd=0.3):
    """Means uniform in [-half, half]^3 (the small single-view workload)."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-half, half, size=(n, 3))
    log_scale = rng.normal(ls_mu, ls_sd, size=(n, 3))
    quat = _random_quats(rng, n)
    opac = rng.normal(0.0, op_sd, size=n)
    sh = rng.normal(0.0, sh_sd, size=(n, 4, 3))
    return _soa(mean, log_scale, quat, opac, sh)


def _uniform_ball(rng, n, radius):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.uniform(0.0, 1.0, size=n) ** (1.0 / 3.0)
    return d * r[:, None]


def make_scene_ball(n, seed, radius=10.0, ls_mu=-3.5, ls_sd=0.5, op_sd=1.5, sh_sd=0.3):
    """Config-1 attribute distributions with means uniform in a ball."""
    rng = np.random.default_rng(seed)
    mean = _uniform_ball(rng, n, radius)
    log_scale = rng.normal(ls_mu, ls_sd, size=(n, 3))
    quat = _random_quats(rng, n)
    opac = rng.normal(0.0, op_sd, size=n)
    sh = rng.normal(0.0, sh_sd, size=(n, 4, 3))
    return _soa(mean, log_scale, quat, opac, sh)


def make_scene_unbounded(n, seed):
    """Unbounded-scene recipe: 70% clustered in a ball of radius 5, 30% on a far shell.

    The ball part is a mixture of 32 Gaussian clusters (centres uniform in a
    ball of radius 4, member offsets N(0, 0.5^2 I), points outside radius 5
    redrawn); the shell part has directions uniform on the sphere and radius
    U[20, 100].  log-scales N(-4, 1), opacity logits N(0, 2), SH1 N(0, 0.3).
    """
    rng = np.random.default_rng(seed)
    n_ball = int(round(0.7 * n))
    n_shell = n - n_ball
    centres = _uniform_ball(rng, 32, 4.0)
    which = rng.integers(0, 32, size=n_ball)
    pts = centres[which] + rng.normal(0.0, 0.5, size=(n_ball, 3))
    for _ in range(64):
        bad = np.linalg.norm(pts, axis=1) > 5.0
        if not bad.any():
            break
        nb = int(bad.sum())
        w2 = rng.integers(0, 32, size=nb)
        pts[bad] = centres[w2] + rng.normal(0.0, 0.5, size=(nb, 3))
    bad = np.linalg.norm(pts, axis=1) > 5.0
    pts[bad] *= (5.0 / np.linalg.norm(pts[bad], axis=1))[:, None]
    d = rng.normal(size=(n_shell, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    shell = d * rng.uniform(20.0, 100.0, size=n_shell)[:, None]
    mean = np.concatenate([pts, shell], axis=0)
    log_scale = rng.normal(-4.0, 1.0, size=(n, 3))
    quat = _random_quats(rng, n)
    opac = rng.normal(0.0, 2.0, size=n)
    sh = rng.normal(0.0, 0.3, size=(n, 4, 3))
    return _soa(mean, log_scale, quat, opac, sh)


def perturb_scene(scene, seed, mean_sd=0.01, opac_sd=0.2):
    """Copy of ``scene`` with means + N(0, mean_sd) and opacity logits + N(0, opac_sd)."""
    rng = np.random.default_rng(seed)
    out = {k: v.copy() for k, v in scene.items()}
    out["mean"] = (out["mean"] + rng.normal(0, mean_sd, size=out["mean"].shape)).astype(np.float32)
    out["opacity_logit"] = (out["opacity_logit"]
                            + rng.normal(0, opac_sd, size=out["opacity_logit"].shape)).astype(np.float32)
    return out


def make_mlp(seed, hidden=MLP_HIDDEN, n_in=MLP_IN):
    """He-normal FP32 master weights; phi head starts near 1, opacity head near sigma(2)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, math.sqrt(2.0 / n_in), size=(hidden, n_in))
    W2 = rng.normal(0, math.sqrt(2.0 / hidden), size=(hidden, hidden))
    w_phi = 0.1 * rng.normal(0, math.sqrt(2.0 / hidden), size=hidden)
    w_o = rng.normal(0, math.sqrt(2.0 / hidden), size=hidden)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(W1=f32(W1), b1=f32(np.zeros(hidden)), W2=f32(W2), b2=f32(np.zeros(hidden)),
                w_phi=f32(w_phi), b_phi=np.float32(1.0), w_o=f32(w_o), b_o=np.float32(2.0))


def make_sortfree_params(n, seed, sigma_range=(0.02, 0.6), beta_range=(0.5, 1.8)):
    """Per-Gaussian (sigma, beta) of the SortFreeGS weighting function w = exp(-sigma d^beta)
    (Eq. 1): float32 arrays drawn uniformly in the given ranges (sigma first, then beta)."""
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(*sigma_range, n).astype(np.float32)
    beta = rng.uniform(*beta_range, n).astype(np.float32)
    return sigma, beta


def with_sh_degree(scene, degree, seed, sd_high=0.1):
    """Copy of a first-order-SH scene with SH of ``degree`` (0..3): degree 0 keeps the DC
    coefficient of each channel; degrees 2 and 3 append coefficients N(0, sd_high) drawn from
    their own stream (so the lower-order ones stay those of the input).  SH planes stay
    coefficient-major (plane 3 k + channel)."""
    if degree not in (0, 1, 2, 3):
        raise ValueError("SH degree must be 0..3")
    out = dict(scene)
    sh = np.asarray(scene["sh"])
    n = sh.shape[1]
    K = (degree + 1) ** 2
    if K <= 4:
        out["sh"] = np.ascontiguousarray(sh[:3 * K], dtype=np.float32)
    else:
        rng = np.random.default_rng([seed, 2])
        extra = rng.normal(0.0, sd_high, size=(3 * (K - 4), n))
        out["sh"] = np.ascontiguousarray(np.concatenate([sh, extra], axis=0), dtype=np.float32)
    return out


MLP_F_WIDTHS = (256, 128, 64)   # the appendix's MLP_f hidden layers


def make_mlp_f(seed, widths=MLP_F_WIDTHS, n_in=MLP_IN):
    """He-normal FP32 master weights of an MLP with ReLU hidden layers of the given widths
    (keys W1, b1, W2, b2, ...); heads as make_mlp (phi near 1, opacity factor near sigma(2))."""
    rng = np.random.default_rng(seed)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    out, prev = {}, n_in
    for k, h in enumerate(widths, start=1):
        out[f"W{k}"] = f32(rng.normal(0, math.sqrt(2.0 / prev), size=(h, prev)))
        out[f"b{k}"] = f32(0.05 * rng.normal(size=h))
        prev = h
    out["w_phi"] = f32(0.1 * rng.normal(0, math.sqrt(2.0 / prev), size=prev))
    out["b_phi"] = np.float32(1.0)
    out["w_o"] = f32(rng.normal(0, math.sqrt(2.0 / prev), size=prev))
    out["b_o"] = np.float32(2.0)
    return out


def circle_poses(n_poses, radius, width, height, f=None, elevation_deg=0.0):
    cams = []
    el = math.radians(elevation_deg)
    for k in range(n_poses):
        az = 2.0 * math.pi * k / n_poses
        eye = (radius * math.cos(el) * math.sin(az), -radius * math.sin(el),
               -radius * math.cos(el) * math.cos(az))
        cams.append(look_at(eye, width=width, height=height, f=f))
    return cams


def _catmull_rom(p0, p1, p2, p3, u):
    return 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u * u
                  + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)


def spline_poses(n_poses, width, height, f=None):
    """Closed Catmull-Rom path through 6 control points around the origin."""
    ctrl = []
    for k in range(6):
        az = math.radians(60.0 * k)
        r = 18.0 if k % 2 == 0 else 24.0
        el = math.radians(0.0 if k % 2 == 0 else 15.0)
        ctrl.append(np.array([r * math.cos(el) * math.sin(az), -r * math.sin(el),
                              -r * math.cos(el) * math.cos(az)]))
    cams = []
    for i in range(n_poses):
        s = 6.0 * i / n_poses
        k = int(s)
        u = s - k
        p = _catmull_rom(ctrl[(k - 1) % 6], ctrl[k % 6], ctrl[(k + 1) % 6], ctrl[(k + 2) % 6], u)
        cams.append(look_at(p, width=width, height=height, f=f))
    return cams


def tiny_scene(n, seed, width=32, height=32, depth=4.0, half=1.0):
    """Small scene + camera for finite-difference and closed-form checks."""
    scene = make_scene_uniform(n, seed, half=half)
    cam = look_at((0.0, 0.0, -depth), width=width, height=height, f=float(width))
    return scene, cam


def make_config(name, seed=0, n=None):
    """Return (scene, cameras, mlp_or_None, tile) for a named workload.

    ``small``   2,000 Gaussians uniform in [-1,1]^3, one 128x128 view, f=128, no MLP.
    ``unbounded`` 1,000,000 Gaussians (clustered ball + far shell), 32 poses on
                a circle of radius 10, 1600x1063, f=1600, MLP on.
    ``large``   3,000,000 Gaussians uniform in a ball of radius 10, 60 spline
                poses, 1920x1080, f=1920, MLP on.
    ``train``   500,000 Gaussians (small-workload attributes), 4 views at 1600x1063.
    ``n`` overrides the Gaussian count (used for reduced-size parity runs).
    """
    if name == "small":
        n = 2000 if n is None else n
        scene = make_scene_uniform(n, seed)
        cam = look_at((0.0, 0.0, -4.0), width=128, height=128, f=128.0)
        return scene, [cam], None, 16
    if name == "unbounded":
        n = 1_000_000 if n is None else n
        scene = make_scene_unbounded(n, seed)
        cams = circle_poses(32, 10.0, 1600, 1063, f=1600.0)
        return scene, cams, make_mlp(seed + 1), 16
    if name == "large":
        n = 3_000_000 if n is None else n
        scene = make_scene_ball(n, seed, radius=10.0)
        cams = spline_poses(60, 1920, 1080, f=1920.0)
        return scene, cams, make_mlp(seed + 1), 16
    if name == "train":
        n = 500_000 if n is None else n
        scene = make_scene_uniform(n, seed)
        cams = circle_poses(4, 4.0, 1600, 1063, f=1600.0)
        return scene, cams, make_mlp(seed + 1), 16
    raise ValueError(f"unknown workload {name!r}")


# ---------------------------------------------------------------------------
# Vector-quantised scenes.  The 20 non-position attributes of a Gaussian are cut into
# NVQ_GROUPS sub-vectors of NVQ_DIM values, each an index into its own codebook of
# NVQ_CODEWORDS rows (see oracle/nvq.py for the layout both sides decode).
NVQ_GROUPS = 5
NVQ_DIM = 4
NVQ_CODEWORDS = 1024


def _attribute_rows(scene):
    """(N, 20) float32 rows [log_scale(3), quat(4), opacity_logit, sh(12)] of a scene."""
    return np.concatenate([scene["log_scale"].T, scene["quat"].T, scene["opacity_logit"][:, None],
                           scene["sh"].T], axis=1).astype(np.float32)


def make_nvq(scene, seed, codewords=NVQ_CODEWORDS):
    """A vector-quantised scene with the positions of ``scene``: every codebook holds the
    sub-vectors of ``codewords`` Gaussians of ``scene`` drawn at random (so each attribute
    keeps the scene's distribution), and every Gaussian draws its five codes uniformly.
    Returns dict(mean [3][N] float32, codes [5][N] uint16, codebooks [5][codewords][4] float32).
    """
    rng = np.random.default_rng(seed)
    rows = _attribute_rows(scene)
    n = rows.shape[0]
    cb = np.empty((NVQ_GROUPS, codewords, NVQ_DIM), np.float32)
    for g in range(NVQ_GROUPS):
        pick = rng.integers(0, n, size=codewords)
        cb[g] = rows[pick, g * NVQ_DIM:(g + 1) * NVQ_DIM]
    codes = rng.integers(0, codewords, size=(NVQ_GROUPS, n)).astype(np.uint16)
    return dict(mean=np.ascontiguousarray(scene["mean"], np.float32), codes=codes, codebooks=cb)
