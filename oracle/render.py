"""FP64 reference of the order-independent Gaussian splatting pass (test infrastructure).

Inputs are the float32 arrays produced by ``mgs_data`` (upcast to float64 here,
so input quantisation is not an error source).  Everything is torch-CPU float64
so that autograd supplies reference gradients.

Steps, in the paper's order:

1. activate the stored attributes (Appendix B: mean, covariance from scale and
   rotation, opacity in [0, 1], SH colour);
2. camera-space position, depth d and the camera-to-Gaussian vector P_i (Sec. 3.1);
3. first-order SH colour (Sec. 3.2 keeps SH degree 1);
4. view-dependent enhancement MLP -> phi, modulating opacity (Eq. 4);
5. depth-aware weight w = phi^2 + phi/d^2 + exp(s_max/d) (Eq. 3);
6. perspective (EWA) projection to a 2D conic (Appendix B: "standard perspective
   camera model"; EWA splatting of Zwicker et al. is the standard one);
7. alpha of a Gaussian at a pixel, alpha = o exp(-1/2 dx^T Sigma'^-1 dx) (Eq. 2);
8. per-pixel composite C = (1-T) sum(c a w)/sum(a w) + T c_bg,
   T = prod(1 - alpha) (Eq. 2);
9. for comparison, front-to-back sorted alpha blending (Eq. 11).
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = [
    "ALPHA_MIN", "ALPHA_MAX", "DILATION", "JAC_CLAMP", "T_STOP", "SH_C0", "SH_C1",
    "AMBIG_LOG", "DEPTH_KEY_ULPS", "POS_ULPS", "to64", "quat_to_rotmat", "activate", "camera_space", "sh1_color",
    "mlp_features", "sh_basis", "sh_color", "enhance", "depth_weight", "ewa_cov2d", "project", "bin_lists",
    "bin_lists_bruteforce", "bin_lists_sorted", "pixel_grid", "eval_pixels_oit", "render_oit",
    "render_sorted", "render", "camera_tensors", "oit_pixel_variants", "ambiguous_gaussians",
]

DT = torch.float64

# Constants (readings of points the paper leaves to the 3DGS convention).
ALPHA_MIN = 1.0 / 255.0   # a Gaussian contributes to a pixel only if its alpha >= 1/255
ALPHA_MAX = 0.99          # alpha is clamped so 1 - alpha stays >= 0.01
DILATION = 0.3            # screen-space low-pass added to the 2D covariance (px^2)
JAC_CLAMP = 1.3           # view-frustum clamp of x/z, y/z used for the EWA Jacobian
T_STOP = 1e-4             # sorted path only: stop once transmittance drops below this
SH_C0 = 0.5 / math.sqrt(math.pi)                  # real SH, l=0
SH_C1 = math.sqrt(3.0) / (2.0 * math.sqrt(math.pi))  # real SH, l=1
AMBIG_LOG = 1e-4          # |ln(a / alpha_min)| below this -> the pair's inclusion is ambiguous
POS_ULPS = 4.0            # float32 error bound of a screen mean, in 2^-24 x the magnitude of its terms
DEPTH_KEY_ULPS = 8.0      # sorted path: float32 error bound of a depth key, in 2^-24 x magnitude


def to64(a, requires_grad=False):
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), dtype=DT).clone()
    if requires_grad:
        t.requires_grad_(True)
    return t


def camera_tensors(cam):
    """Camera fields as float64 tensors/floats (the camera is a ``mgs_data.Camera``)."""
    return dict(R=to64(cam.R), t=to64(cam.t), fx=float(cam.fx), fy=float(cam.fy),
                cx=float(cam.cx), cy=float(cam.cy), W=int(cam.width), H=int(cam.height),
                near=float(cam.near))


# --------------------------------------------------------------------------
# Step 1 -- activation of the stored attributes (Appendix B).
# --------------------------------------------------------------------------
def quat_to_rotmat(q):
    """Rotation matrix of unit quaternions q = (w, x, y, z), shape (N, 4) -> (N, 3, 3)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r00 = 1 - 2 * (y * y + z * z)
    r01 = 2 * (x * y - w * z)
    r02 = 2 * (x * z + w * y)
    r10 = 2 * (x * y + w * z)
    r11 = 1 - 2 * (x * x + z * z)
    r12 = 2 * (y * z - w * x)
    r20 = 2 * (x * z - w * y)
    r21 = 2 * (y * z + w * x)
    r22 = 1 - 2 * (x * x + y * y)
    return torch.stack([torch.stack([r00, r01, r02], -1),
                        torch.stack([r10, r11, r12], -1),
                        torch.stack([r20, r21, r22], -1)], -2)


def activate(params):
    """Scale s = exp(log_scale), unit rotation, covariance R S S^T R^T, opacity sigma(logit).

    ``params`` holds (N, k)-shaped float64 tensors: mean (N,3), log_scale (N,3),
    quat (N,4), opacity_logit (N,), sh (N,4,3).  A zero quaternion is rejected.
    """
    s = torch.exp(params["log_scale"])
    qn = params["quat"].norm(dim=1, keepdim=True)
    if bool((qn == 0).any()):
        raise ValueError("zero quaternion")
    q = params["quat"] / qn
    Rq = quat_to_rotmat(q)
    Sigma = Rq @ torch.diag_embed(s * s) @ Rq.transpose(1, 2)
    o = torch.sigmoid(params["opacity_logit"])
    return dict(s=s, q=q, Rq=Rq, Sigma=Sigma, o=o)


# --------------------------------------------------------------------------
# Step 2 -- camera space, depth and the camera-to-Gaussian vector (Sec. 3.1).
# --------------------------------------------------------------------------
def camera_space(mean, cam):
    """x_c = R mu + t; depth d = x_c.z; centre t_v = -R^T t; P = (mu - t_v)/|mu - t_v|."""
    R, t = cam["R"], cam["t"]
    x_c = mean @ R.T + t
    d = x_c[:, 2]
    t_v = -(R.T @ t)
    v = mean - t_v
    P = v / v.norm(dim=1, keepdim=True)
    return x_c, d, P


# --------------------------------------------------------------------------
# Step 3 -- first-order SH colour (Sec. 3.2; real SH basis, 3DGS sign convention).
# --------------------------------------------------------------------------
def sh1_color(P, sh):
    """c = max(0, 1/2 + C0 Y0 + C1 (-P_y Y1 + P_z Y2 - P_x Y3)); sh is (N, 4, 3)."""
    x, y, z = P[:, 0:1], P[:, 1:2], P[:, 2:3]
    c = 0.5 + SH_C0 * sh[:, 0] + SH_C1 * (-y * sh[:, 1] + z * sh[:, 2] - x * sh[:, 3])
    return torch.clamp(c, min=0.0)


def sh_basis(P, degree):
    """Orthonormal real SH up to ``degree`` (0..3) at unit directions P: (N, (degree+1)^2),
    coefficient l^2 + l + m for order m = -l..l, with the sign (-1)^m on odd m (the l = 1 terms
    are then -C1 y, C1 z, -C1 x, as in sh1_color)."""
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    one = torch.ones_like(x)
    out = [SH_C0 * one]
    if degree >= 1:
        out += [-SH_C1 * y, SH_C1 * z, -SH_C1 * x]
    if degree >= 2:
        a, b, c = 0.5 * math.sqrt(15 / math.pi), 0.25 * math.sqrt(5 / math.pi), 0.25 * math.sqrt(15 / math.pi)
        out += [a * x * y, -a * y * z, b * (3 * z * z - 1), -a * x * z, c * (x * x - y * y)]
    if degree >= 3:
        a = 0.25 * math.sqrt(35 / (2 * math.pi))
        b = 0.5 * math.sqrt(105 / math.pi)
        c = 0.25 * math.sqrt(21 / (2 * math.pi))
        d = 0.25 * math.sqrt(7 / math.pi)
        e = 0.25 * math.sqrt(105 / math.pi)
        out += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (5 * z * z - 1), d * z * (5 * z * z - 3),
                -c * x * (5 * z * z - 1), e * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=1)


SH_DEGREE_OF = {1: 0, 4: 1, 9: 2, 16: 3}


def sh_color(P, sh):
    """c = max(0, 1/2 + sum_k Y_k(P) sh_k) for sh (N, K, 3), K = (degree+1)^2 of degree 0..3
    (Table 3's SH-order variants); degree 1 is sh1_color itself."""
    K = sh.shape[1]
    if K == 4:
        return sh1_color(P, sh)
    Y = sh_basis(P, SH_DEGREE_OF[K])
    return torch.clamp(0.5 + (Y[:, :, None] * sh).sum(dim=1), min=0.0)


# --------------------------------------------------------------------------
# Step 4 -- neural view-dependent enhancement (Eq. 4).
# --------------------------------------------------------------------------
def mlp_features(P, s, q, sh):
    """MLP input [P_i, s_i, r_i, Y_i]: 3 + 3 + 4 + 12 = 22 values per Gaussian.  Y_i is the
    degree <= 1 block of the SH coefficients (the first four of each channel; zeros for a
    degree-0 model)."""
    n, K = sh.shape[0], sh.shape[1]
    Y = sh[:, :4] if K >= 4 else torch.cat([sh, torch.zeros(n, 4 - K, 3, dtype=sh.dtype)], dim=1)
    return torch.cat([P, s, q, Y.reshape(n, 12)], dim=1)


def bf16_round(x):
    """Round to bfloat16 (round-to-nearest-even) the way a float32 kernel does: via float32.

    The rounding models the precision of the kernel's MFMA inputs; for gradients it
    is the identity (straight-through), so the gradient itself is never rounded.
    """
    r = x.detach().to(torch.float32).to(torch.bfloat16).to(DT)
    return x + (r - x).detach() if x.requires_grad else r


def enhance(x, mlp, bf16=False):
    """F = MLP_f(x), phi = ReLU(MLP_phi(F)), m = sigmoid(MLP_o(F)) (Eq. 4).

    MLP_f is the chain of ReLU layers W1, b1, W2, b2, ... (every ``Wk`` present, in
    order): two layers of 64 (the benchmark shape) or the appendix's three of 256, 128
    and 64.  ``mlp`` holds float64 tensors Wk (h_k, h_{k-1}), bk, w_phi (h_L,), b_phi,
    w_o (h_L,), b_o.  With ``bf16`` the inputs of every product (x, the weights, the
    hidden activations and F) are rounded to bfloat16 first and the products are
    summed in float64, standing in for BF16-in / FP32-accumulate.
    """
    h = bf16_round(x) if bf16 else x
    k = 1
    while f"W{k}" in mlp:
        W = bf16_round(mlp[f"W{k}"]) if bf16 else mlp[f"W{k}"]
        h = torch.relu(h @ W.T + mlp[f"b{k}"])
        if bf16:
            h = bf16_round(h)
        k += 1
    wp, wo = mlp["w_phi"], mlp["w_o"]
    if bf16:
        wp, wo = bf16_round(wp), bf16_round(wo)
    phi = torch.relu(h @ wp + mlp["b_phi"])
    m = torch.sigmoid(h @ wo + mlp["b_o"])
    return phi, m


# --------------------------------------------------------------------------
# Step 5 -- depth-aware weight (Eq. 3).
# --------------------------------------------------------------------------
# Eq. 3 and the two ablations of it in the paper's ablation table (Table 3): "without
# depth" read as d = 1 in Eq. 3, "without scale" as Eq. 3 without its exp(s_max / d) term.
# WEIGHT_SORTFREE is the weighting function of the SortFreeGS composite the paper starts
# from (Eq. 1, Sec. 2): w(d_i) = exp(-sigma_i d_i^beta_i), with per-Gaussian sigma_i, beta_i.
WEIGHT_EQ3, WEIGHT_NO_DEPTH, WEIGHT_NO_SCALE, WEIGHT_SORTFREE = 0, 1, 2, 3


def depth_weight(phi, d, s, mode=WEIGHT_EQ3, sortfree=None):
    """w = phi^2 + phi / d^2 + exp(s_max / d); s_max = largest activated scale (Eq. 3),
    or an ablation: mode WEIGHT_NO_DEPTH puts d = 1, WEIGHT_NO_SCALE drops the last term;
    or mode WEIGHT_SORTFREE: w = exp(-sigma d^beta) (Eq. 1) with ``sortfree`` = (sigma, beta),
    two (N,) tensors (phi and the scale play no part)."""
    s_max = s.max(dim=1).values
    if mode == WEIGHT_EQ3:
        return phi * phi + phi / (d * d) + torch.exp(s_max / d)
    if mode == WEIGHT_NO_DEPTH:
        return phi * phi + phi + torch.exp(s_max)
    if mode == WEIGHT_NO_SCALE:
        return phi * phi + phi / (d * d)
    if mode == WEIGHT_SORTFREE:
        if sortfree is None:
            raise ValueError("WEIGHT_SORTFREE needs (sigma, beta)")
        sigma, beta = sortfree
        return torch.exp(-sigma * d ** beta)
    raise ValueError(f"unknown weight mode {mode}")


# --------------------------------------------------------------------------
# Step 6 -- EWA projection of the 3D covariance (Appendix B, perspective camera).
# --------------------------------------------------------------------------
def ewa_cov2d(x_c, Sigma, cam):
    """Sigma' = J W Sigma W^T J^T + 0.3 I with J the Jacobian of (x,y,z) -> (fx x/z, fy y/z).

    J is taken at the camera-space point with x/z, y/z clamped to 1.3x the
    half field of view (so off-screen Gaussians stay well conditioned).
    """
    fx, fy = cam["fx"], cam["fy"]
    z = x_c[:, 2]
    lim_x = JAC_CLAMP * (0.5 * cam["W"]) / fx
    lim_y = JAC_CLAMP * (0.5 * cam["H"]) / fy
    tx = torch.clamp(x_c[:, 0] / z, -lim_x, lim_x) * z
    ty = torch.clamp(x_c[:, 1] / z, -lim_y, lim_y) * z
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * tx / (z * z)], -1),
                     torch.stack([zero, fy / z, -fy * ty / (z * z)], -1)], -2)  # (N,2,3)
    M = J @ cam["R"]                                                          # (N,2,3)
    cov = M @ Sigma @ M.transpose(1, 2)
    cov = cov + DILATION * torch.eye(2, dtype=DT)
    return cov


def project(params, cam, phi=None, m=None, tile=16, weight_mode=WEIGHT_EQ3, sortfree=None):
    """Per-Gaussian preprocessing: everything the per-pixel blend needs.

    Returns float64 tensors: mean2d (N,2), cov2d (N,2,2), conic (N,3) =
    (A, B, C) of Sigma'^-1, color (N,3), o_eff (N,), w (N,), depth (N,), and
    integer results: visible (N,) bool, rect (N,4) int64 = (tx0, ty0, tx1, ty1)
    inclusive tile coordinates, n_tiles (N,) int64.  Culled Gaussians have
    n_tiles = 0 and rect = 0.  ``weight_mode`` / ``sortfree`` select w (depth_weight);
    with tile = 1 the rect is the pixel range itself.

    Culling: depth <= near; o_eff < alpha_min; an empty pixel range.  The rect is
    the set of tiles touched by the pixel centres inside the exact bounding box
    of {alpha >= alpha_min} = {q <= 2 ln(o_eff / alpha_min)}.
    """
    act = activate(params)
    x_c, d, P = camera_space(params["mean"], cam)
    color = sh_color(P, params["sh"])
    n = d.shape[0]
    if phi is None:
        phi = torch.ones(n, dtype=DT)
    if m is None:
        m = torch.ones(n, dtype=DT)
    o_eff = act["o"] * m
    front = d > cam["near"]
    # culled points get depth 1 in the weight (keeps d^beta real; they never reach the blend)
    w = depth_weight(phi, torch.where(front, d, torch.ones_like(d)) if weight_mode == WEIGHT_SORTFREE else d,
                     act["s"], weight_mode, sortfree)
    # Keep the projection finite for culled points (they never reach the blend).
    d_safe = torch.where(front, d, torch.ones_like(d))
    x_safe = torch.cat([x_c[:, :2], d_safe[:, None]], dim=1)
    cov = ewa_cov2d(x_safe, act["Sigma"], cam)
    a, b, c = cov[:, 0, 0], cov[:, 0, 1], cov[:, 1, 1]
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], dim=1)
    mean2d = torch.stack([cam["fx"] * x_safe[:, 0] / d_safe + cam["cx"],
                          cam["fy"] * x_safe[:, 1] / d_safe + cam["cy"]], dim=1)
    with torch.no_grad():
        vis = front & (o_eff >= ALPHA_MIN)
        k = 2.0 * torch.log(torch.clamp(o_eff, min=ALPHA_MIN) / ALPHA_MIN)
        ex = torch.sqrt(k * a)
        ey = torch.sqrt(k * c)
        mx, my = mean2d[:, 0], mean2d[:, 1]
        W, H = cam["W"], cam["H"]
        i0 = torch.ceil(mx - ex - 0.5).clamp(0, W - 1 + 1)
        i1 = torch.floor(mx + ex - 0.5).clamp(-1, W - 1)
        j0 = torch.ceil(my - ey - 0.5).clamp(0, H - 1 + 1)
        j1 = torch.floor(my + ey - 0.5).clamp(-1, H - 1)
        vis = vis & (i0 <= i1) & (j0 <= j1)
        i0, i1, j0, j1 = (v.to(torch.int64) for v in (i0, i1, j0, j1))
        rect = torch.stack([torch.div(i0, tile, rounding_mode="floor"),
                            torch.div(j0, tile, rounding_mode="floor"),
                            torch.div(i1, tile, rounding_mode="floor"),
                            torch.div(j1, tile, rounding_mode="floor")], dim=1)
        rect = torch.where(vis[:, None], rect, torch.zeros_like(rect))
        n_tiles = torch.where(vis, (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1),
                              torch.zeros_like(rect[:, 0]))
    # magnitude of the terms of d = R_z . mu + t_z (scales the float32 error of a depth key)
    mu_abs = params["mean"].detach().abs()
    depth_mag = (mu_abs @ cam["R"][2].abs()) + abs(float(cam["t"][2]))
    # float32 error bound of the screen mean f x_c / d + c per axis: POS_ULPS units of 2^-24 times
    # the magnitude of its terms (x_c = R_x . mu + t_x summed in magnitude, then the offset c)
    with torch.no_grad():
        dabs = d_safe.detach().abs()
        mag_x = cam["fx"] * ((mu_abs @ cam["R"][0].abs()) + abs(float(cam["t"][0]))) / dabs + abs(cam["cx"])
        mag_y = cam["fy"] * ((mu_abs @ cam["R"][1].abs()) + abs(float(cam["t"][1]))) / dabs + abs(cam["cy"])
        pos_err = POS_ULPS * 2.0 ** -24 * torch.maximum(mag_x, mag_y)
    return dict(mean2d=mean2d, cov2d=cov, conic=conic, color=color, o_eff=o_eff, w=w,
                depth=d, depth_mag=depth_mag, pos_err=pos_err, visible=vis, rect=rect, n_tiles=n_tiles, phi=phi, m=m,
                tiles_x=(cam["W"] + tile - 1) // tile, tiles_y=(cam["H"] + tile - 1) // tile,
                tile=tile)


# --------------------------------------------------------------------------
# Tile lists (ascending Gaussian index per tile; no depth order).
# --------------------------------------------------------------------------
def bin_lists(rect, n_tiles, tiles_x, tiles_y):
    """Per-tile lists of the Gaussians whose rect covers the tile, ascending index.

    Returns (tile_offsets (T+1,), gids (P,)) as int64 tensors, tiles row-major
    t = ty * tiles_x + tx.  Pairs are enumerated Gaussian by Gaussian and put
    in tile order with a stable sort (a library primitive).
    """
    rect = torch.as_tensor(rect, dtype=torch.int64)
    n_tiles = torch.as_tensor(n_tiles, dtype=torch.int64)
    T = tiles_x * tiles_y
    gid = torch.repeat_interleave(torch.arange(rect.shape[0]), n_tiles)
    if gid.numel() == 0:
        return torch.zeros(T + 1, dtype=torch.int64), gid
    start = torch.cumsum(n_tiles, 0) - n_tiles
    k = torch.arange(gid.numel()) - start[gid]
    wdt = rect[gid, 2] - rect[gid, 0] + 1
    tx = rect[gid, 0] + k % wdt
    ty = rect[gid, 1] + torch.div(k, wdt, rounding_mode="floor")
    tile = ty * tiles_x + tx
    order = torch.sort(tile, stable=True).indices
    gids = gid[order]
    counts = torch.bincount(tile, minlength=T)
    offsets = torch.zeros(T + 1, dtype=torch.int64)
    offsets[1:] = torch.cumsum(counts, 0)
    return offsets, gids


def bin_lists_sorted(rect, n_tiles, depth, tiles_x, tiles_y):
    """Per-tile lists ordered by (depth, index) -- the sorted comparison path (Eq. 11).

    ``depth`` is taken as given (the caller passes the precision the sort key
    has).  Returns (tile_offsets, gids) like ``bin_lists``.
    """
    offs, gids = bin_lists(rect, n_tiles, tiles_x, tiles_y)
    depth = torch.as_tensor(np.asarray(depth), dtype=DT)
    out = gids.clone()
    for t in range(tiles_x * tiles_y):
        a, b = int(offs[t]), int(offs[t + 1])
        if b - a > 1:
            seg = gids[a:b]
            out[a:b] = seg[torch.sort(depth[seg], stable=True).indices]
    return offs, out


def bin_lists_bruteforce(rect, n_tiles, tiles_x, tiles_y):
    """O(N * T) enumeration of the same lists (pins ``bin_lists`` on small inputs)."""
    rect = np.asarray(rect)
    n_tiles = np.asarray(n_tiles)
    offsets = [0]
    gids = []
    for ty in range(tiles_y):
        for tx in range(tiles_x):
            for g in range(rect.shape[0]):
                if n_tiles[g] > 0 and rect[g, 0] <= tx <= rect[g, 2] and rect[g, 1] <= ty <= rect[g, 3]:
                    gids.append(g)
            offsets.append(len(gids))
    return np.asarray(offsets, np.int64), np.asarray(gids, np.int64)


# --------------------------------------------------------------------------
# Steps 7-8 -- per-pixel alpha and the order-independent composite (Eq. 2, Eq. 3).
# --------------------------------------------------------------------------
def pixel_grid(W, H):
    """Pixel centres (i + 1/2, j + 1/2) in row-major order, shape (H*W, 2)."""
    jj, ii = torch.meshgrid(torch.arange(H, dtype=DT), torch.arange(W, dtype=DT), indexing="ij")
    return torch.stack([ii.reshape(-1) + 0.5, jj.reshape(-1) + 0.5], dim=1)


def _alpha(pix, mean2d, conic, o_eff):
    """a = o exp(-q/2), q = dx^T Sigma'^-1 dx; (n_pix, n_g) matrices."""
    dx = pix[:, 0:1] - mean2d[None, :, 0]
    dy = pix[:, 1:2] - mean2d[None, :, 1]
    q = conic[None, :, 0] * dx * dx + 2.0 * conic[None, :, 1] * dx * dy + conic[None, :, 2] * dy * dy
    return o_eff[None, :] * torch.exp(-0.5 * q)


def _ambiguous(pix, proj, idx, a, alpha_min):
    """Pairs whose side of the alpha cut a float32 evaluation may not reproduce (n_pix, n_g):
    |ln(a / alpha_min)| < AMBIG_LOG + |grad_pixel ln a|_1 pos_err, where ln a moves by
    |A dx| per pixel of screen-mean error and pos_err bounds that error for the Gaussian
    (proj["pos_err"], zero when absent)."""
    band = AMBIG_LOG
    pos = proj.get("pos_err")
    near = (a > alpha_min * math.exp(-0.05)) & (a < alpha_min * math.exp(0.05))
    if pos is None or not bool(near.any()):
        return (a > alpha_min * math.exp(-band)) & (a < alpha_min * math.exp(band))
    conic, mean2d = proj["conic"][idx].detach(), proj["mean2d"][idx].detach()
    dx = pix[:, 0:1] - mean2d[None, :, 0]
    dy = pix[:, 1:2] - mean2d[None, :, 1]
    grad = (conic[None, :, 0] * dx + conic[None, :, 1] * dy).abs() + (conic[None, :, 1] * dx + conic[None, :, 2] * dy).abs()
    width = band + grad * pos[idx].detach()[None, :]
    return near & (torch.log(a / alpha_min).abs() < width)


def eval_pixels_oit(pix, proj, idx, alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, track_ambiguous=False):
    """Sums of Eq. 2 for the pixels ``pix`` over the Gaussians ``idx``.

    Returns N (n_pix,3) = sum c alpha w, D = sum alpha w, T = prod(1 - alpha) over
    the contributors (alpha >= alpha_min, alpha clamped at alpha_max), and the
    contributor count.  With ``track_ambiguous`` also returns, per pixel, up to
    two ambiguous pairs (see _ambiguous) as their contributions
    (c a w, a w, 1 - a, nominally_in) and the number of ambiguous pairs.
    """
    idx = torch.as_tensor(idx, dtype=torch.int64)
    mean2d, conic, o_eff = proj["mean2d"][idx], proj["conic"][idx], proj["o_eff"][idx]
    color, w = proj["color"][idx], proj["w"][idx]
    a = _alpha(pix, mean2d, conic, o_eff)
    inc = a >= alpha_min
    al = torch.clamp(a, max=alpha_max)
    al = torch.where(inc, al, torch.zeros_like(al))
    aw = al * w[None, :]
    N = aw @ color
    D = aw.sum(dim=1)
    T = torch.prod(1.0 - al, dim=1)
    cnt = inc.sum(dim=1)
    if not track_ambiguous:
        return N, D, T, cnt
    with torch.no_grad():
        amb = _ambiguous(pix, proj, idx, a.detach(), alpha_min)
        n_amb = amb.sum(dim=1)
        n = a.shape[0]
        amb_list = [dict(has=torch.zeros(n, dtype=torch.bool), cw=torch.zeros(n, 3, dtype=DT),
                         aw=torch.zeros(n, dtype=DT), one_minus=torch.ones(n, dtype=DT),
                         nominal=torch.zeros(n, dtype=torch.bool)) for _ in range(2)]
        rows = torch.nonzero(n_amb > 0).reshape(-1)       # the pixels with an ambiguous pair
        if rows.numel() == 0:
            return N, D, T, cnt, amb_list, n_amb
        a_r, inc_r = a[rows], inc[rows]
        al_raw = torch.clamp(a_r, max=alpha_max)
        # the first two ambiguous pairs of each such pixel, in list order
        score = amb[rows].to(torch.int64) * torch.arange(a.shape[1], 0, -1)[None, :]
        for k in range(2):
            j = torch.argmax(score, dim=1)
            has = score.gather(1, j[:, None])[:, 0] > 0
            alj = al_raw.gather(1, j[:, None])[:, 0]
            wj = w[j]
            e = amb_list[k]
            e["has"][rows] = has
            e["cw"][rows] = color[j] * (alj * wj)[:, None]
            e["aw"][rows] = alj * wj
            e["one_minus"][rows] = 1.0 - alj
            e["nominal"][rows] = inc_r.gather(1, j[:, None])[:, 0]
            score = score.scatter(1, j[:, None], 0)
    return N, D, T, cnt, amb_list, n_amb


def ambiguous_gaussians(proj, cam, lists=None, alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX):
    """Gaussians with at least one pixel pair whose side of a cut float32 may not reproduce:
    the alpha_min cut (see _ambiguous) or the alpha_max clamp (same band around alpha_max).
    The render of such a Gaussian's pixels is admissible either way, and its gradient has a
    term (the pair's) that float32 may include or not.  Per tile over the tile lists (by
    default the oracle's own).  Returns a bool tensor (N,)."""
    W, H = cam["W"], cam["H"]
    if lists is None:
        lists = bin_lists(proj["rect"], proj["n_tiles"], proj["tiles_x"], proj["tiles_y"])
    offs, gids = (torch.as_tensor(np.asarray(v), dtype=torch.int64) for v in lists)
    pix = pixel_grid(W, H)
    B = proj["tile"]
    out = torch.zeros(proj["o_eff"].shape[0], dtype=torch.bool)
    with torch.no_grad():
        for t in range(proj["tiles_x"] * proj["tiles_y"]):
            g = gids[offs[t]:offs[t + 1]]
            if g.numel() == 0:
                continue
            tx, ty = t % proj["tiles_x"], t // proj["tiles_x"]
            ii = torch.arange(tx * B, min(W, tx * B + B))
            jj = torch.arange(ty * B, min(H, ty * B + B))
            pp = pix[(jj[:, None] * W + ii[None, :]).reshape(-1)]
            a = _alpha(pp, proj["mean2d"][g].detach(), proj["conic"][g].detach(), proj["o_eff"][g].detach())
            amb = _ambiguous(pp, proj, g, a, alpha_min) | _ambiguous(pp, proj, g, a, alpha_max)
            out[g[amb.any(0)]] = True
    return out


def _composite(N, D, T, bg, w_bg=None):
    """C = (1 - T) N / D + T c_bg, and C = c_bg where no Gaussian contributes (Eq. 2).

    With ``w_bg`` (a float >= 0) the SortFreeGS composite of Eq. 1 instead:
    C = (c_bg w_bg + N) / (w_bg + D), T unused, and C = c_bg where w_bg + D = 0.
    F = N / D (0 where D = 0) is returned in both cases."""
    has = D > 0
    Dsafe = torch.where(has, D, torch.ones_like(D))
    F = torch.where(has[:, None], N / Dsafe[:, None], torch.zeros_like(N))
    if w_bg is not None:
        den = D + w_bg
        pos = den > 0
        C = (N + w_bg * bg[None, :]) / torch.where(pos, den, torch.ones_like(den))[:, None]
        return torch.where(pos[:, None], C, bg[None, :].expand_as(C)), F
    C = (1.0 - T)[:, None] * F + T[:, None] * bg[None, :]
    return torch.where(has[:, None], C, bg[None, :].expand_as(C)), F


def oit_pixel_variants(N, D, T, amb_list, bg, w_bg=None):
    """Images for every way the (at most two) ambiguous pairs of a pixel may fall.

    Returns (4, n_pix, 3): variant v toggles ambiguous pair k when bit k of v
    is set (pixels with fewer ambiguous pairs repeat their nominal result).
    ``w_bg``: composite of Eq. 1 instead of Eq. 2 (see _composite).
    """
    outs = []
    for v in range(4):
        Nv, Dv, Tv = N.clone(), D.clone(), T.clone()
        for k, e in enumerate(amb_list):
            tog = e["has"] & bool(v >> k & 1)
            sign = torch.where(e["nominal"], -1.0, 1.0).to(DT)
            s = torch.where(tog, sign, torch.zeros_like(sign))
            Nv = Nv + s[:, None] * e["cw"]
            Dv = Dv + s * e["aw"]
            fac = torch.where(tog & e["nominal"], 1.0 / e["one_minus"],
                              torch.where(tog, e["one_minus"], torch.ones_like(e["one_minus"])))
            Tv = Tv * fac
        Dv = torch.where(Dv.abs() < 1e-12, torch.zeros_like(Dv), Dv)
        C, _ = _composite(Nv, Dv, Tv, bg, w_bg)
        outs.append(C)
    return torch.stack(outs)


def render_oit(proj, cam, bg, mode="brute", lists=None, chunk=1 << 22, variants=False,
               alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, w_bg=None):
    """Image (3, H, W) of Eq. 2 (or, with ``w_bg``, of Eq. 1's composite).

    ``mode='brute'`` evaluates every pixel against every visible Gaussian;
    ``mode='binned'`` evaluates each tile's pixels against that tile's list
    (``lists`` = (tile_offsets, gids); by default the oracle's own lists).
    Also returns aux (5, H, W) = (F_r, F_g, F_b, D, T) with F = N / D.
    With ``variants`` returns (4, 3, H, W) admissible images and the count of
    pixels with more than two ambiguous pairs.
    """
    W, H = cam["W"], cam["H"]
    bg = torch.as_tensor(np.asarray(bg, np.float64), dtype=DT)
    pix = pixel_grid(W, H)
    n_pix = pix.shape[0]
    N = torch.zeros(n_pix, 3, dtype=DT)
    D = torch.zeros(n_pix, dtype=DT)
    T = torch.ones(n_pix, dtype=DT)
    amb_store = [dict(has=torch.zeros(n_pix, dtype=torch.bool), cw=torch.zeros(n_pix, 3, dtype=DT),
                      aw=torch.zeros(n_pix, dtype=DT), one_minus=torch.ones(n_pix, dtype=DT),
                      nominal=torch.zeros(n_pix, dtype=torch.bool)) for _ in range(2)]
    n_amb = torch.zeros(n_pix, dtype=torch.int64)

    def run(pix_idx, gidx):
        nonlocal N, D, T, n_amb
        if len(gidx) == 0 or len(pix_idx) == 0:
            return
        res = eval_pixels_oit(pix[pix_idx], proj, gidx, alpha_min, alpha_max, track_ambiguous=variants)
        if variants:
            n_, d_, t_, _, amb, na = res
            for k in range(2):
                for key in ("has", "cw", "aw", "one_minus", "nominal"):
                    amb_store[k][key][pix_idx] = amb[k][key]
            n_amb[pix_idx] = na
        else:
            n_, d_, t_, _ = res
        if n_.requires_grad or d_.requires_grad or t_.requires_grad:
            # out of place, so autograd sees each tile's sums as a separate input
            N = N.index_put((pix_idx,), n_)
            D = D.index_put((pix_idx,), d_)
            T = T.index_put((pix_idx,), t_)
        else:
            N[pix_idx] = n_
            D[pix_idx] = d_
            T[pix_idx] = t_

    if mode == "brute":
        gidx = torch.nonzero(proj["visible"]).reshape(-1)
        step = max(1, chunk // max(1, len(gidx)))
        for p0 in range(0, n_pix, step):
            run(torch.arange(p0, min(n_pix, p0 + step)), gidx)
    elif mode == "binned":
        if lists is None:
            lists = bin_lists(proj["rect"], proj["n_tiles"], proj["tiles_x"], proj["tiles_y"])
        offs, gids = (torch.as_tensor(np.asarray(v), dtype=torch.int64) for v in lists)
        B = proj["tile"]
        for t in range(proj["tiles_x"] * proj["tiles_y"]):
            g = gids[offs[t]:offs[t + 1]]
            if g.numel() == 0:
                continue
            tx, ty = t % proj["tiles_x"], t // proj["tiles_x"]
            ii = torch.arange(tx * B, min(W, tx * B + B))
            jj = torch.arange(ty * B, min(H, ty * B + B))
            pidx = (jj[:, None] * W + ii[None, :]).reshape(-1)
            run(pidx, g)
    else:
        raise ValueError(mode)
    C, F = _composite(N, D, T, bg, w_bg)
    img = C.T.reshape(3, H, W)
    aux = torch.cat([F.T, D[None], T[None]], dim=0).reshape(5, H, W)
    if not variants:
        return img, aux
    V = oit_pixel_variants(N, D, T, amb_store, bg, w_bg)      # (4, n_pix, 3)
    V = V.permute(0, 2, 1).reshape(4, 3, H, W)
    flagged = int((n_amb > 2).sum())
    return img, aux, V, flagged


# --------------------------------------------------------------------------
# Step 9 -- sorted front-to-back alpha blending, the comparison path (Eq. 11).
# --------------------------------------------------------------------------
def _sorted_pixels(pix, proj, order, bg, alpha_min, alpha_max, t_stop, want_flags):
    """Eq. 11 for the pixels ``pix`` over the Gaussians ``order`` (already in (depth, index)
    order): returns the colours (n_pix, 3) and, with ``want_flags``, the fragility flags."""
    a = _alpha(pix, proj["mean2d"][order], proj["conic"][order], proj["o_eff"][order])
    inc = a >= alpha_min
    al = torch.where(inc, torch.clamp(a, max=alpha_max), torch.zeros_like(a))
    one_m = 1.0 - al
    Tin = torch.cumprod(torch.cat([torch.ones(pix.shape[0], 1, dtype=DT), one_m[:, :-1]], 1), 1)
    live = Tin >= t_stop
    contrib = (al * Tin * live) @ proj["color"][order]
    Tfin = torch.prod(torch.where(live, one_m, torch.ones_like(one_m)), dim=1)
    out = contrib + Tfin[:, None] * bg[None, :]
    if not want_flags:
        return out, None
    with torch.no_grad():
        dep = proj["depth"][order].detach()
        amb = _ambiguous(pix, proj, order, a, alpha_min).any(1)
        near_stop = ((Tin / t_stop - 1.0).abs() < 1e-3).any(1)
        # Depth ties a float32 sort key cannot order: two contributors composited before the
        # stop whose depths differ by no more than the float32 evaluation error of the key,
        # bounded by DEPTH_KEY_ULPS units of 2^-24 times the magnitude of the terms of
        # d = R_z . mu + t_z (proj["depth_mag"]).  Contributors behind the stop do not count.
        mag = proj["depth_mag"][order].detach()
        live_c = inc & (Tin >= t_stop * (1.0 - 1e-3))
        # ``order`` is ascending in depth, so each live contributor's predecessor among the live
        # ones is the running maximum of the live depths before it
        prev, pidx = torch.cummax(torch.where(live_c, dep[None, :].expand_as(a), torch.full_like(a, -math.inf)), 1)
        prev, pidx = prev[:, :-1], pidx[:, :-1]
        gap = dep[None, 1:] - prev
        tol = DEPTH_KEY_ULPS * 2.0 ** -24 * (mag[None, 1:] + mag[pidx])
        tie = (live_c[:, 1:] & torch.isfinite(prev) & (gap <= tol)).any(1)
        flags = amb | near_stop | tie
    return out, flags


def render_sorted(proj, cam, bg, chunk=1 << 21, alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX,
                  t_stop=T_STOP, return_flags=False, mode="brute", lists=None):
    """C = sum_k c_k alpha_k T_k + T_K c_bg over contributors sorted by (depth, index).

    T_k = prod_{j<k}(1 - alpha_j).  A contributor is composited only while the
    transmittance before it is still >= t_stop (early stop).  With
    ``return_flags`` also returns a per-pixel flag marking results that a
    float32 implementation may legitimately order or stop differently (near
    depth ties among contributors, transmittance within 0.1% of t_stop, or an
    ambiguous alpha cut).

    ``mode='brute'`` sorts every visible Gaussian for every pixel; ``mode='binned'``
    evaluates each tile's pixels over that tile's list only (``lists`` = (tile_offsets,
    gids), by default the oracle's own), sorted by (depth, index): the same result,
    since a Gaussian outside a tile's list has alpha < alpha_min on all its pixels.
    """
    W, H = cam["W"], cam["H"]
    bg = torch.as_tensor(np.asarray(bg, np.float64), dtype=DT)
    pix = pixel_grid(W, H)
    n_pix = pix.shape[0]
    out = bg[None, :].repeat(n_pix, 1)
    flags = torch.zeros(n_pix, dtype=torch.bool)
    if mode == "brute":
        gidx = torch.nonzero(proj["visible"]).reshape(-1)
        # depth order, ties by Gaussian index (stable sort of an index-ordered array)
        order = gidx[torch.sort(proj["depth"][gidx].detach(), stable=True).indices]
        step = max(1, chunk // max(1, len(order)))
        for p0 in range(0, n_pix, step):
            pi = torch.arange(p0, min(n_pix, p0 + step))
            o, f = _sorted_pixels(pix[pi], proj, order, bg, alpha_min, alpha_max, t_stop, return_flags)
            out[pi] = o
            if return_flags:
                flags[pi] = f
    elif mode == "binned":
        if lists is None:
            lists = bin_lists(proj["rect"], proj["n_tiles"], proj["tiles_x"], proj["tiles_y"])
        offs, gids = (torch.as_tensor(np.asarray(v), dtype=torch.int64) for v in lists)
        B = proj["tile"]
        depth = proj["depth"].detach()
        for t in range(proj["tiles_x"] * proj["tiles_y"]):
            g = gids[offs[t]:offs[t + 1]]
            if g.numel() == 0:
                continue
            g = torch.sort(g).values                                   # index order, then
            order = g[torch.sort(depth[g], stable=True).indices]      # stable by depth
            tx, ty = t % proj["tiles_x"], t // proj["tiles_x"]
            ii = torch.arange(tx * B, min(W, tx * B + B))
            jj = torch.arange(ty * B, min(H, ty * B + B))
            pidx = (jj[:, None] * W + ii[None, :]).reshape(-1)
            o, f = _sorted_pixels(pix[pidx], proj, order, bg, alpha_min, alpha_max, t_stop, return_flags)
            out[pidx] = o
            if return_flags:
                flags[pidx] = f
    else:
        raise ValueError(mode)
    img = out.T.reshape(3, H, W)
    if return_flags:
        return img, flags.reshape(H, W)
    return img


# --------------------------------------------------------------------------
# Whole pass.
# --------------------------------------------------------------------------
def scene_params(scene, requires_grad=False):
    """Float32 SoA scene arrays -> (N, k) float64 tensors (leaves if requires_grad)."""
    n = scene["mean"].shape[1]
    p = dict(mean=to64(np.asarray(scene["mean"]).T, requires_grad),
             log_scale=to64(np.asarray(scene["log_scale"]).T, requires_grad),
             quat=to64(np.asarray(scene["quat"]).T, requires_grad),
             opacity_logit=to64(scene["opacity_logit"], requires_grad),
             sh=to64(np.asarray(scene["sh"]).T.reshape(n, np.asarray(scene["sh"]).shape[0] // 3, 3),
                     requires_grad))
    return p


def mlp_params(mlp, requires_grad=False):
    return {k: to64(np.asarray(v), requires_grad) for k, v in mlp.items()}


def render(scene, cam, mlp=None, bg=(0.0, 0.0, 0.0), bf16=False, mode="brute", tile=16,
           params=None, mparams=None, sorted_path=False, weight_mode=WEIGHT_EQ3, sortfree=None, w_bg=None):
    """Enhance -> project -> (bin) -> blend for one view; returns (image, aux, proj).
    ``sortfree`` = (sigma, beta) arrays and ``w_bg`` select Eq. 1 (with WEIGHT_SORTFREE)."""
    camt = camera_tensors(cam)
    p = scene_params(scene) if params is None else params
    phi = m = None
    if mlp is not None or mparams is not None:
        mp = mlp_params(mlp) if mparams is None else mparams
        act = activate(p)
        _, _, P = camera_space(p["mean"], camt)
        x = mlp_features(P, act["s"], act["q"], p["sh"])
        phi, m = enhance(x, mp, bf16=bf16)
    if sortfree is not None:
        sortfree = tuple(to64(np.asarray(v)) for v in sortfree)
    proj = project(p, camt, phi, m, tile, weight_mode, sortfree)
    if sorted_path:
        return render_sorted(proj, camt, bg), None, proj
    img, aux = render_oit(proj, camt, bg, mode=mode, w_bg=w_bg)
    return img, aux, proj


__all__ += ["scene_params", "mlp_params", "bf16_round", "WEIGHT_EQ3", "WEIGHT_NO_DEPTH", "WEIGHT_NO_SCALE",
            "WEIGHT_SORTFREE"]
