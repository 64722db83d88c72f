"""Pins of the FP64 oracle against facts other than itself.

Each test fixes one part of the oracle with a closed form, a textbook special
case, an invariant of the mathematics, or brute force on a tiny input, so that
a plausible mistake (dropped term, wrong sign or index, transposed operand)
fails at least one of them.  Passages: Eq. 2 / Eq. 3 / Eq. 4 (Sec. 3.1),
Eq. 11 (Appendix B).
"""
import math

import numpy as np
import pytest
import torch

import mgs_data
import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")


def _cam_identity(W=32, H=32, f=32.0, z=4.0):
    return mgs_data.look_at((0.0, 0.0, -z), width=W, height=H, f=f)


def _one_gaussian(mean=(0, 0, 0), log_scale=(-2, -2, -2), quat=(1, 0, 0, 0), logit=0.0, sh=None):
    sh = np.zeros((4, 3)) if sh is None else np.asarray(sh, np.float64)
    return dict(mean=np.asarray(mean, np.float32).reshape(3, 1),
                log_scale=np.asarray(log_scale, np.float32).reshape(3, 1),
                quat=np.asarray(quat, np.float32).reshape(4, 1),
                opacity_logit=np.asarray([logit], np.float32),
                sh=np.asarray(sh, np.float32).reshape(1, 12).T.copy())


def _concat(*scenes):
    return {k: np.concatenate([s[k] for s in scenes], axis=-1) for k in scenes[0]}


# ---------------------------------------------------------------- rotation
def test_quat_rotation_textbook_and_invariants():
    th = 0.7
    q = torch.tensor([[math.cos(th / 2), 0, 0, math.sin(th / 2)]], dtype=torch.float64)
    R = O.quat_to_rotmat(q)[0]
    ref = torch.tensor([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]],
                       dtype=torch.float64)
    assert torch.allclose(R, ref, atol=1e-15)
    # about x
    qx = torch.tensor([[math.cos(th / 2), math.sin(th / 2), 0, 0]], dtype=torch.float64)
    refx = torch.tensor([[1, 0, 0], [0, math.cos(th), -math.sin(th)], [0, math.sin(th), math.cos(th)]],
                        dtype=torch.float64)
    assert torch.allclose(O.quat_to_rotmat(qx)[0], refx, atol=1e-15)
    rng = np.random.default_rng(1)
    qs = torch.tensor(rng.normal(size=(64, 4)))
    qs = qs / qs.norm(dim=1, keepdim=True)
    Rs = O.quat_to_rotmat(qs)
    eye = torch.eye(3, dtype=torch.float64).expand(64, 3, 3)
    assert torch.allclose(Rs @ Rs.transpose(1, 2), eye, atol=1e-13)
    assert torch.allclose(torch.linalg.det(Rs), torch.ones(64, dtype=torch.float64), atol=1e-13)
    assert torch.allclose(O.quat_to_rotmat(-qs), Rs, atol=1e-15)
    # composition: R(q1 * q2) = R(q1) R(q2) (Hamilton product written out here)
    q1, q2 = qs[:32], qs[32:]
    w1, x1, y1, z1 = q1.T
    w2, x2, y2, z2 = q2.T
    prod = torch.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)
    assert torch.allclose(O.quat_to_rotmat(prod), Rs[:32] @ Rs[32:], atol=1e-13)


def test_activate_isotropic_and_sigmoid():
    sc = _one_gaussian(log_scale=(-1.5, -1.5, -1.5), quat=(0.3, -0.2, 0.9, 0.1), logit=0.0)
    act = O.activate(O.scene_params(sc))
    s = math.exp(-1.5)
    assert torch.allclose(act["Sigma"][0], (s * s) * torch.eye(3, dtype=torch.float64), atol=1e-15)
    assert abs(float(act["o"][0]) - 0.5) < 1e-15
    with pytest.raises(ValueError):
        O.activate(O.scene_params(_one_gaussian(quat=(0, 0, 0, 0))))


# ---------------------------------------------------------------- SH colour
C0_TEXTBOOK = 0.28209479177387814   # Y_0^0 = 1 / (2 sqrt(pi))
C1_TEXTBOOK = 0.4886025119029199    # |Y_1^m| normalisation = sqrt(3 / (4 pi))


def test_sh1_color_axes():
    rng = np.random.default_rng(3)
    sh = torch.tensor(rng.normal(0, 0.3, size=(6, 4, 3)))
    P = torch.tensor([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                     dtype=torch.float64)
    c = O.sh1_color(P, sh)
    base = 0.5 + C0_TEXTBOOK * sh[:, 0]
    exp = torch.stack([base[0] - C1_TEXTBOOK * sh[0, 3], base[1] + C1_TEXTBOOK * sh[1, 3],
                       base[2] - C1_TEXTBOOK * sh[2, 1], base[3] + C1_TEXTBOOK * sh[3, 1],
                       base[4] + C1_TEXTBOOK * sh[4, 2], base[5] - C1_TEXTBOOK * sh[5, 2]])
    assert torch.allclose(c, exp.clamp(min=0), atol=1e-15)
    # clamp at zero
    neg = torch.zeros((1, 4, 3), dtype=torch.float64)
    neg[0, 0] = -5.0
    assert float(O.sh1_color(P[:1], neg).max()) == 0.0


# ---------------------------------------------------------------- SH orders 0-3 (Table 3 variants)
def _unit_dirs(n, seed):
    P = np.random.default_rng(seed).normal(size=(n, 3))
    return P / np.linalg.norm(P, axis=1, keepdims=True)


def test_sh_basis_is_the_real_harmonics_of_scipy_with_odd_m_negated():
    """Degrees 0..3 against scipy's complex harmonics turned real (standard real form, no
    Condon-Shortley phase), times (-1)^m on odd m: the convention that gives -C1 y, C1 z, -C1 x."""
    from scipy.special import sph_harm_y
    P = _unit_dirs(40, 3)
    theta, phi = np.arccos(P[:, 2]), np.arctan2(P[:, 1], P[:, 0])
    Y = O.sh_basis(torch.tensor(P), 3).numpy()
    for l in range(4):
        for m in range(-l, l + 1):
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * sph_harm_y(l, m, theta, phi).real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * sph_harm_y(l, -m, theta, phi).imag
            else:
                ref = sph_harm_y(l, 0, theta, phi).real
            sign = -1.0 if m % 2 else 1.0
            assert np.allclose(Y[:, l * l + l + m], sign * ref, atol=1e-12, rtol=0), (l, m)


def test_sh_basis_is_orthonormal_on_the_sphere():
    """Gauss-Legendre in cos(theta) x uniform phi (exact for these polynomial degrees)."""
    from scipy.special import roots_legendre
    u, wu = roots_legendre(12)
    ph = np.arange(24) * (2 * math.pi / 24)
    ct, pp = np.meshgrid(u, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    P = np.stack([st * np.cos(pp), st * np.sin(pp), ct], -1).reshape(-1, 3)
    w = (wu[:, None] * np.full(24, 2 * math.pi / 24)[None]).reshape(-1)
    Y = O.sh_basis(torch.tensor(P), 3).numpy()
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_sh_color_of_every_order_and_the_features_it_feeds():
    rng = np.random.default_rng(4)
    P = torch.tensor(_unit_dirs(30, 5))
    sh3 = torch.tensor(rng.normal(0, 0.3, size=(30, 16, 3)))
    # order 1 through the general basis is sh1_color; order 3 by an explicit sum per coefficient
    Y = O.sh_basis(P, 3)
    c1 = torch.clamp(0.5 + sum(Y[:, k, None] * sh3[:, k] for k in range(4)), min=0.0)
    assert torch.allclose(O.sh1_color(P, sh3[:, :4]), c1, atol=1e-14)
    c3 = torch.clamp(0.5 + sum(Y[:, k, None] * sh3[:, k] for k in range(16)), min=0.0)
    assert torch.allclose(O.sh_color(P, sh3), c3, atol=1e-14)
    c0 = O.sh_color(P, sh3[:, :1])
    assert torch.allclose(c0, torch.clamp(0.5 + O.SH_C0 * sh3[:, 0], min=0.0).expand(30, 3), atol=1e-15)
    # the MLP sees the degree <= 1 block: equal for orders 1-3, zero-padded for order 0
    s = torch.ones(30, 3, dtype=torch.float64)
    q = torch.ones(30, 4, dtype=torch.float64)
    f1 = O.mlp_features(P, s, q, sh3[:, :4])
    assert torch.equal(O.mlp_features(P, s, q, sh3), f1) and torch.equal(O.mlp_features(P, s, q, sh3[:, :9]), f1)
    f0 = O.mlp_features(P, s, q, sh3[:, :1])
    assert torch.equal(f0[:, :13], f1[:, :13]) and float(f0[:, 13:].abs().max()) == 0.0


# ---------------------------------------------------------------- weight (Eq. 3)
def test_depth_weight_closed_form():
    phi = torch.tensor([1.0, 0.0, 2.5], dtype=torch.float64)
    d = torch.tensor([2.0, 4.0, 0.5], dtype=torch.float64)
    s = torch.tensor([[0.5, 0.1, 0.2], [0.3, 0.9, 0.2], [0.1, 0.1, 0.4]], dtype=torch.float64)
    w = O.depth_weight(phi, d, s)
    exp = [1.0 + 1.0 / 4.0 + math.exp(0.25), math.exp(0.9 / 4.0), 6.25 + 2.5 / 0.25 + math.exp(0.8)]
    assert np.allclose(w.numpy(), exp, rtol=1e-15, atol=0)


def test_weight_ablations_drop_exactly_their_dependence():
    """Table 3's Eq. 3 ablations: "without depth" leaves w independent of the camera distance,
    "without scale" independent of the Gaussians' scales; Eq. 3 itself depends on both."""
    scene = mgs_data.make_scene_uniform(300, 11)
    p = O.scene_params(scene)
    near, far = (O.camera_tensors(mgs_data.look_at((0.0, 0.0, -z), width=64, height=64)) for z in (4.0, 6.5))
    with torch.no_grad():
        w = {(m, c): O.project(p, cam, weight_mode=m)["w"] for m in (0, 1, 2) for c, cam in (("n", near), ("f", far))}
    assert torch.equal(w[(O.WEIGHT_NO_DEPTH, "n")], w[(O.WEIGHT_NO_DEPTH, "f")])
    assert not torch.allclose(w[(O.WEIGHT_EQ3, "n")], w[(O.WEIGHT_EQ3, "f")])
    assert not torch.allclose(w[(O.WEIGHT_NO_SCALE, "n")], w[(O.WEIGHT_NO_SCALE, "f")])
    big = dict(scene)
    big["log_scale"] = scene["log_scale"] + np.float32(0.7)
    pb = O.scene_params(big)
    with torch.no_grad():
        wb = {m: O.project(pb, near, weight_mode=m)["w"] for m in (0, 2)}
    assert torch.equal(wb[O.WEIGHT_NO_SCALE], w[(O.WEIGHT_NO_SCALE, "n")])
    assert not torch.allclose(wb[O.WEIGHT_EQ3], w[(O.WEIGHT_EQ3, "n")])
    # the three differ pairwise on the same view
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert not torch.allclose(w[(a, "n")], w[(b, "n")])


def test_weight_eq3_at_unit_depth_is_the_no_depth_ablation():
    """Every Gaussian on the plane z = 0 seen from (0, 0, -1): d = 1, where Eq. 3 and its
    "without depth" reading coincide; the "without scale" one is 1 (= exp 0) lower."""
    scene = mgs_data.make_scene_uniform(200, 12, half=0.3)
    scene = dict(scene)
    mean = scene["mean"].copy()
    mean[2] = 0.0
    scene["mean"] = mean
    p = O.scene_params(scene)
    cam = O.camera_tensors(mgs_data.look_at((0.0, 0.0, -1.0), width=64, height=64))
    with torch.no_grad():
        d = O.camera_space(p["mean"], cam)[1]
        assert torch.equal(d, torch.ones_like(d))
        w0, w1, w2 = (O.project(p, cam, weight_mode=m)["w"] for m in (0, 1, 2))
    assert torch.equal(w0, w1)
    s_max = O.activate(p)["s"].max(dim=1).values
    assert torch.allclose(w0 - w2, torch.exp(s_max), rtol=1e-14, atol=0)


# ---------------------------------------------------------------- EWA projection
def test_ewa_closed_form_on_axis():
    f, z = 100.0, 5.0
    cam = O.camera_tensors(mgs_data.look_at((0, 0, -z), width=64, height=64, f=f))
    # isotropic, arbitrary rotation
    sc = _one_gaussian(log_scale=(-2, -2, -2), quat=(0.2, 0.5, -0.7, 0.1))
    pr = O.project(O.scene_params(sc), cam)
    s = math.exp(-2)
    v = (f * s / z) ** 2 + 0.3
    assert torch.allclose(pr["cov2d"][0], v * torch.eye(2, dtype=torch.float64), rtol=1e-13)
    assert torch.allclose(pr["mean2d"][0], torch.tensor([32.0, 32.0], dtype=torch.float64))
    # axis-aligned anisotropic
    sc = _one_gaussian(log_scale=(-1, -2.5, -3), quat=(1, 0, 0, 0))
    pr = O.project(O.scene_params(sc), cam)
    ref = torch.diag(torch.tensor([(f * math.exp(-1) / z) ** 2 + 0.3, (f * math.exp(-2.5) / z) ** 2 + 0.3],
                                  dtype=torch.float64))
    assert torch.allclose(pr["cov2d"][0], ref, rtol=1e-13)
    # conic is the inverse
    A, B, C = pr["conic"][0]
    M = torch.tensor([[A, B], [B, C]])
    assert torch.allclose(M @ pr["cov2d"][0], torch.eye(2, dtype=torch.float64), atol=1e-12)


def _screen_map(cam, x):
    xc = cam["R"] @ x + cam["t"]
    return torch.stack([cam["fx"] * xc[0] / xc[2] + cam["cx"], cam["fy"] * xc[1] / xc[2] + cam["cy"]])


def test_ewa_matches_finite_difference_linearisation():
    """Off-axis Gaussians seen from a rotated camera: Sigma' = J_fd Sigma J_fd^T + 0.3 I."""
    cam_o = mgs_data.look_at((3.0, -1.0, -6.0), target=(0.3, 0.2, 0.1), width=200, height=150, f=180.0)
    cam = O.camera_tensors(cam_o)
    sc = mgs_data.make_scene_uniform(12, seed=5, half=0.8)
    p = O.scene_params(sc)
    pr = O.project(p, cam)
    act = O.activate(p)
    h = 1e-5
    for g in range(12):
        mu = p["mean"][g].detach()
        J = torch.zeros(2, 3, dtype=torch.float64)
        for k in range(3):
            e = torch.zeros(3, dtype=torch.float64)
            e[k] = h
            J[:, k] = (_screen_map(cam, mu + e) - _screen_map(cam, mu - e)) / (2 * h)
        # only valid where the frustum clamp is inactive
        xc = cam["R"] @ mu + cam["t"]
        if abs(float(xc[0] / xc[2])) > 1.3 * 100 / 180 or abs(float(xc[1] / xc[2])) > 1.3 * 75 / 180:
            continue
        ref = J @ act["Sigma"][g] @ J.T + 0.3 * torch.eye(2, dtype=torch.float64)
        assert torch.allclose(pr["cov2d"][g], ref, rtol=1e-7, atol=1e-9), g
        assert torch.allclose(pr["mean2d"][g], _screen_map(cam, mu), atol=1e-10)


def test_support_extent_matches_sampled_ellipse():
    """e_x, e_y are the extreme x, y of the ellipse {q = 2 ln(o/alpha_min)} (sampled)."""
    cam = O.camera_tensors(mgs_data.look_at((0, 0, -3), width=96, height=80, f=90.0))
    sc = mgs_data.make_scene_uniform(20, seed=7, half=0.6, ls_mu=-2.5)
    pr = O.project(O.scene_params(sc), cam)
    th = torch.linspace(0, 2 * math.pi, 200001, dtype=torch.float64)
    for g in range(20):
        if not bool(pr["visible"][g]):
            continue
        k = 2 * math.log(float(pr["o_eff"][g]) / (1 / 255))
        ev, evec = torch.linalg.eigh(pr["cov2d"][g])
        pts = evec @ torch.stack([torch.sqrt(k * ev[0]) * torch.cos(th), torch.sqrt(k * ev[1]) * torch.sin(th)])
        ex, ey = float(pts[0].max()), float(pts[1].max())
        a, c = float(pr["cov2d"][g][0, 0]), float(pr["cov2d"][g][1, 1])
        assert abs(math.sqrt(k * a) - ex) < 1e-6 * (1 + ex)
        assert abs(math.sqrt(k * c) - ey) < 1e-6 * (1 + ey)


def _alpha_bruteforce(pr, g, W, H):
    """alpha of Gaussian g at every pixel centre, written out per pixel (tiny images only)."""
    mx, my = float(pr["mean2d"][g, 0]), float(pr["mean2d"][g, 1])
    A, B, C = (float(v) for v in pr["conic"][g])
    o = float(pr["o_eff"][g])
    out = np.zeros((H, W))
    for j in range(H):
        for i in range(W):
            dx, dy = i + 0.5 - mx, j + 0.5 - my
            out[j, i] = o * math.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + C * dy * dy))
    return out


def test_rect_covers_every_contributing_pixel():
    W, H, B = 48, 40, 16
    cam = O.camera_tensors(mgs_data.look_at((0, 0, -3), width=W, height=H, f=48.0))
    sc = mgs_data.make_scene_uniform(40, seed=11, half=0.9, ls_mu=-2.8)
    pr = O.project(O.scene_params(sc), cam, tile=B)
    seen = 0
    for g in range(40):
        a = _alpha_bruteforce(pr, g, W, H)
        jj, ii = np.nonzero(a >= 1 / 255)
        if not bool(pr["visible"][g]):
            assert len(ii) == 0 or float(pr["depth"][g]) <= 0.2
            continue
        seen += 1
        r = pr["rect"][g].tolist()
        assert len(ii) > 0 or True
        for i, j in zip(ii, jj):
            assert r[0] <= i // B <= r[2] and r[1] <= j // B <= r[3]
        assert int(pr["n_tiles"][g]) == (r[2] - r[0] + 1) * (r[3] - r[1] + 1)
    assert seen > 10


# ---------------------------------------------------------------- lists
def test_bin_lists_equal_bruteforce():
    rng = np.random.default_rng(2)
    tx, ty, n = 7, 5, 300
    x0 = rng.integers(0, tx, n)
    y0 = rng.integers(0, ty, n)
    x1 = np.minimum(tx - 1, x0 + rng.integers(0, 3, n))
    y1 = np.minimum(ty - 1, y0 + rng.integers(0, 3, n))
    rect = np.stack([x0, y0, x1, y1], 1)
    nt = (x1 - x0 + 1) * (y1 - y0 + 1)
    nt[rng.random(n) < 0.2] = 0          # culled
    rect[nt == 0] = 0
    o1, g1 = O.bin_lists(rect, nt, tx, ty)
    o2, g2 = O.bin_lists_bruteforce(rect, nt, tx, ty)
    assert np.array_equal(o1.numpy(), o2) and np.array_equal(g1.numpy(), g2)
    o3, g3 = O.bin_lists(np.zeros((0, 4), np.int64), np.zeros(0, np.int64), tx, ty)
    assert o3.numel() == tx * ty + 1 and int(o3.sum()) == 0 and g3.numel() == 0


# ---------------------------------------------------------------- blend (Eq. 2)
def test_single_isotropic_gaussian_closed_form():
    W = H = 32
    f, z = 32.0, 4.0
    cam = O.camera_tensors(_cam_identity(W, H, f, z))
    sh = np.zeros((4, 3))
    sh[0] = [0.4, -0.2, 0.1]
    sh[2] = [0.3, 0.1, -0.5]
    ls = -1.6
    sc = _one_gaussian(log_scale=(ls, ls, ls), quat=(0.3, 0.1, 0.8, -0.2), logit=1.2, sh=sh)
    bg = np.array([0.1, 0.6, 0.3])
    img, aux = O.render_oit(O.project(O.scene_params(sc), cam), cam, bg)
    s = math.exp(float(np.float32(ls)))         # inputs are stored as float32
    var = (f * s / z) ** 2 + 0.3
    o = 1 / (1 + math.exp(-float(np.float32(1.2))))
    sh32 = sh.astype(np.float32).astype(np.float64)
    c = np.maximum(0, 0.5 + C0_TEXTBOOK * sh32[0] + C1_TEXTBOOK * sh32[2])  # P = +z
    ref = np.zeros((3, H, W))
    for j in range(H):
        for i in range(W):
            r2 = (i + 0.5 - 16) ** 2 + (j + 0.5 - 16) ** 2
            a = o * math.exp(-0.5 * r2 / var)
            al = min(a, 0.99) if a >= 1 / 255 else 0.0
            ref[:, j, i] = al * c + (1 - al) * bg
    assert np.abs(img.numpy() - ref).max() < 1e-12


def test_empty_scene_is_background():
    cam = O.camera_tensors(_cam_identity(24, 20))
    empty = {k: v[..., :0] for k, v in _one_gaussian().items()}
    bg = np.array([0.2, 0.3, 0.9])
    img, aux = O.render_oit(O.project(O.scene_params(empty), cam), cam, bg)
    assert np.allclose(img.numpy(), bg[:, None, None])
    assert float(aux[3].abs().max()) == 0.0 and float((aux[4] - 1).abs().max()) == 0.0
    # every Gaussian behind the camera
    sc = _one_gaussian(mean=(0, 0, -10))
    pr = O.project(O.scene_params(sc), cam)
    assert not bool(pr["visible"][0]) and int(pr["n_tiles"][0]) == 0
    img2, _ = O.render_oit(pr, cam, bg)
    assert np.allclose(img2.numpy(), bg[:, None, None])


def _small(n=60, seed=4, W=40, H=36):
    sc = mgs_data.make_scene_uniform(n, seed, half=0.9, ls_mu=-2.6)
    cam = O.camera_tensors(mgs_data.look_at((0.2, -0.1, -3.5), width=W, height=H, f=44.0))
    return sc, cam


def test_permutation_invariance():
    sc, cam = _small()
    bg = np.array([0.3, 0.1, 0.7])
    img, aux = O.render_oit(O.project(O.scene_params(sc), cam), cam, bg)
    perm = np.random.default_rng(0).permutation(sc["mean"].shape[1])
    scp = {k: v[..., perm] for k, v in sc.items()}
    img2, _ = O.render_oit(O.project(O.scene_params(scp), cam), cam, bg)
    assert float((img - img2).abs().max()) < 1e-12
    assert float(img.std()) > 1e-3          # the scene is not trivially empty


def test_weight_scale_invariance_and_constant_colour():
    sc, cam = _small()
    bg = np.array([0.3, 0.1, 0.7])
    pr = O.project(O.scene_params(sc), cam)
    img, aux = O.render_oit(pr, cam, bg)
    pr2 = dict(pr)
    pr2["w"] = pr["w"] * 8.0
    img2, _ = O.render_oit(pr2, cam, bg)
    assert float((img - img2).abs().max()) < 1e-13
    # all colours equal -> C = (1 - T) c + T c_bg
    pr3 = dict(pr)
    c = torch.tensor([0.25, 0.5, 0.9], dtype=torch.float64)
    pr3["color"] = c.expand_as(pr["color"]).clone()
    img3, aux3 = O.render_oit(pr3, cam, bg)
    T = aux3[4]
    ref = (1 - T)[None] * c[:, None, None] + T[None] * torch.tensor(bg)[:, None, None]
    assert float((img3 - ref).abs().max()) < 1e-13


def test_duplicate_gaussian_keeps_F_and_squares_T():
    sc, cam = _small(n=30)
    pr = O.project(O.scene_params(sc), cam)
    _, aux = O.render_oit(pr, cam, np.zeros(3))
    dup = {k: np.concatenate([v, v], axis=-1) for k, v in sc.items()}
    _, aux2 = O.render_oit(O.project(O.scene_params(dup), cam), cam, np.zeros(3))
    has = aux[3] > 0
    assert float((aux2[:3] - aux[:3])[:, has].abs().max()) < 1e-12
    assert float((aux2[4] - aux[4] ** 2).abs().max()) < 1e-13
    assert float((aux2[3] - 2 * aux[3]).abs().max()) < 1e-10


def test_opacity_to_zero_gives_background():
    sc, cam = _small(n=30)
    sc = dict(sc)
    sc["opacity_logit"] = np.full_like(sc["opacity_logit"], -40.0)
    bg = np.array([0.5, 0.25, 0.125])
    img, _ = O.render_oit(O.project(O.scene_params(sc), cam), cam, bg)
    assert np.allclose(img.numpy(), bg[:, None, None], atol=0)


def test_binned_equals_bruteforce():
    sc, cam = _small(n=120, W=56, H=44)
    pr = O.project(O.scene_params(sc), cam, tile=16)
    bg = np.array([0.3, 0.1, 0.7])
    a, aux_a = O.render_oit(pr, cam, bg, mode="brute")
    b, aux_b = O.render_oit(pr, cam, bg, mode="binned")
    assert float((a - b).abs().max()) < 1e-13 and float((aux_a - aux_b).abs().max()) < 1e-12
    pr8 = O.project(O.scene_params(sc), cam, tile=8)
    c, _ = O.render_oit(pr8, cam, bg, mode="binned")
    assert float((a - c).abs().max()) < 1e-13


def test_mirror_symmetry():
    """Reflect the scene in x = 0 (camera on the axis): the image mirrors left-right."""
    sc, _ = _small(n=50)
    cam = O.camera_tensors(_cam_identity(40, 30, 40.0, 3.5))
    m = {k: v.copy() for k, v in sc.items()}
    m["mean"][0] *= -1
    m["quat"][2] *= -1          # R' = M R M  <=>  (w, x, -y, -z)
    m["quat"][3] *= -1
    m["sh"][9:12] *= -1          # colour term -P_x Y3 keeps its value
    bg = np.array([0.3, 0.1, 0.7])
    a, _ = O.render_oit(O.project(O.scene_params(sc), cam), cam, bg)
    b, _ = O.render_oit(O.project(O.scene_params(m), cam), cam, bg)
    assert float((a - torch.flip(b, dims=[2])).abs().max()) < 1e-12


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_rigid_motion_invariance():
    """Rotate the world and the camera together (SH l=1 rotated too): same image."""
    sc, _ = _small(n=50)
    cam_o = mgs_data.look_at((0.5, -0.3, -3.5), width=40, height=36, f=44.0)
    ax = np.array([0.3, -0.8, 0.5])
    ax /= np.linalg.norm(ax)
    th = 0.9
    qQ = np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * ax])
    Q = O.quat_to_rotmat(torch.tensor(qQ[None]))[0].numpy()
    m = {k: v.astype(np.float64).copy() for k, v in sc.items()}
    m["mean"] = Q @ m["mean"]
    m["quat"] = np.stack([_quat_mul(qQ, m["quat"][:, i]) for i in range(m["quat"].shape[1])], 1)
    sh = m["sh"].reshape(4, 3, -1)               # [k][ch][n]
    v = np.stack([-sh[3], -sh[1], sh[2]])         # colour = 1/2 + C0 Y0 + C1 v . P
    v2 = np.einsum("ij,jcn->icn", Q, v)
    sh[3], sh[1], sh[2] = -v2[0], -v2[1], v2[2]
    m["sh"] = sh.reshape(12, -1)
    cam2 = dict(O.camera_tensors(cam_o))
    cam2["R"] = cam2["R"] @ torch.tensor(Q).T
    bg = np.array([0.3, 0.1, 0.7])
    p1 = O.scene_params(sc)
    p2 = {k: torch.as_tensor(np.asarray(m[k]).T if k != "sh" else np.asarray(m[k]).T.reshape(-1, 4, 3),
                             dtype=torch.float64) for k in ("mean", "log_scale", "quat", "sh")}
    p2["opacity_logit"] = p1["opacity_logit"]
    a, _ = O.render_oit(O.project(p1, O.camera_tensors(cam_o)), O.camera_tensors(cam_o), bg)
    b, _ = O.render_oit(O.project(p2, cam2), cam2, bg)
    assert float((a - b).abs().max()) < 1e-9


# ---------------------------------------------------------------- sorted path (Eq. 11)
def test_sorted_equals_oit_for_one_and_disjoint_gaussians():
    cam = O.camera_tensors(_cam_identity(48, 32, 48.0, 4.0))
    sc = _concat(_one_gaussian(mean=(-0.8, 0, 0), log_scale=(-3, -3, -3), logit=2.0),
                 _one_gaussian(mean=(0.0, 0.1, 0.5), log_scale=(-3, -2.9, -3), logit=0.5),
                 _one_gaussian(mean=(0.8, -0.2, -0.5), log_scale=(-3.1, -3, -3), logit=4.0))
    pr = O.project(O.scene_params(sc), cam)
    bg = np.array([0.2, 0.4, 0.6])
    a, _ = O.render_oit(pr, cam, bg)
    b = O.render_sorted(pr, cam, bg)
    assert float((a - b).abs().max()) < 1e-14


def test_sorted_two_gaussians_front_to_back():
    """Two co-centred Gaussians at different depths: C = a1 c1 + (1-a1) a2 c2 + (1-a1)(1-a2) bg."""
    W = H = 16
    f = 16.0
    cam = O.camera_tensors(_cam_identity(W, H, f, 4.0))
    sh1 = np.zeros((4, 3))
    sh1[0] = [1.0, -1.0, 0.0]
    sh2 = np.zeros((4, 3))
    sh2[0] = [-1.0, 1.0, 0.5]
    near = _one_gaussian(mean=(0, 0, -1.0), log_scale=(-1.5,) * 3, logit=0.3, sh=sh1)
    far = _one_gaussian(mean=(0, 0, 1.0), log_scale=(-1.2,) * 3, logit=1.5, sh=sh2)
    bg = np.array([0.1, 0.2, 0.3])
    for order in ((far, near), (near, far)):
        pr = O.project(O.scene_params(_concat(*order)), cam)
        img = O.render_sorted(pr, cam, bg).numpy()
        c1 = np.maximum(0, 0.5 + C0_TEXTBOOK * sh1[0])
        c2 = np.maximum(0, 0.5 + C0_TEXTBOOK * sh2[0])
        for (i, j) in ((8, 8), (5, 9), (2, 2)):
            r2 = (i + 0.5 - 8) ** 2 + (j + 0.5 - 8) ** 2
            f32 = lambda v: float(np.float32(v))     # inputs are stored as float32
            v1 = (f * math.exp(f32(-1.5)) / 3.0) ** 2 + 0.3
            v2 = (f * math.exp(f32(-1.2)) / 5.0) ** 2 + 0.3
            a1 = (1 / (1 + math.exp(-f32(0.3)))) * math.exp(-0.5 * r2 / v1)
            a2 = (1 / (1 + math.exp(-f32(1.5)))) * math.exp(-0.5 * r2 / v2)
            a1 = min(a1, 0.99) if a1 >= 1 / 255 else 0
            a2 = min(a2, 0.99) if a2 >= 1 / 255 else 0
            ref = a1 * c1 + (1 - a1) * a2 * c2 + (1 - a1) * (1 - a2) * bg
            assert np.abs(img[:, j, i] - ref).max() < 1e-13


def test_sorted_early_stop():
    """Stacked opaque Gaussians: compositing stops once transmittance < 1e-4."""
    cam = O.camera_tensors(_cam_identity(8, 8, 8.0, 4.0))
    layers = []
    for k in range(4):
        sh = np.zeros((4, 3))
        sh[0] = [float(k), 0.0, 0.0]
        layers.append(_one_gaussian(mean=(0, 0, 0.2 * k), log_scale=(1.0,) * 3, logit=30.0, sh=sh))
    pr = O.project(O.scene_params(_concat(*layers)), cam)
    img = O.render_sorted(pr, cam, np.array([0.0, 0.0, 0.0])).numpy()
    # each layer has alpha ~0.99 near the centre: T = 1, .01, 1e-4(-), ... -> only two layers
    c = [0.5 + C0_TEXTBOOK * k for k in range(4)]
    a = float(pr["o_eff"][0]) * math.exp(-0.5 * 0.0)
    a = min(a, 0.99)
    # the centre pixel has small but non-zero offset; use the composite rule with two live layers
    # T_in for layer 2 = (1 - a0)(1 - a1) < 1e-4 -> stops
    assert img[0, 4, 4] < 0.5 + C0_TEXTBOOK * 1 + 1e-6
    assert img[0, 4, 4] > 0.99 * c[0] - 1e-6


# ---------------------------------------------------------------- MLP (Eq. 4)
def _mlp64(seed=3):
    return O.mlp_params(mgs_data.make_mlp(seed))


def test_mlp_matches_torch_linear_layers():
    mp = _mlp64()
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.normal(size=(50, 22)))
    phi, m = O.enhance(x, mp)
    l1 = torch.nn.Linear(22, 64).double()
    l2 = torch.nn.Linear(64, 64).double()
    hp = torch.nn.Linear(64, 1).double()
    ho = torch.nn.Linear(64, 1).double()
    with torch.no_grad():
        l1.weight.copy_(mp["W1"]); l1.bias.copy_(mp["b1"])
        l2.weight.copy_(mp["W2"]); l2.bias.copy_(mp["b2"])
        hp.weight.copy_(mp["w_phi"][None]); hp.bias.copy_(mp["b_phi"].reshape(1))
        ho.weight.copy_(mp["w_o"][None]); ho.bias.copy_(mp["b_o"].reshape(1))
        Fm = torch.relu(l2(torch.relu(l1(x))))
        assert torch.allclose(phi, torch.relu(hp(Fm))[:, 0], atol=1e-14)
        assert torch.allclose(m, torch.sigmoid(ho(Fm))[:, 0], atol=1e-14)
    assert float(m.min()) > 0 and float(m.max()) < 1 and float(phi.min()) >= 0


def test_mlp_hidden_permutation_and_init():
    mp = _mlp64()
    rng = np.random.default_rng(1)
    x = torch.tensor(rng.normal(size=(40, 22)))
    phi, m = O.enhance(x, mp)
    p1 = torch.tensor(rng.permutation(64))
    p2 = torch.tensor(rng.permutation(64))
    mq = dict(mp)
    mq["W1"] = mp["W1"][p1]
    mq["b1"] = mp["b1"][p1]
    mq["W2"] = mp["W2"][p2][:, p1]
    mq["b2"] = mp["b2"][p2]
    mq["w_phi"] = mp["w_phi"][p2]
    mq["w_o"] = mp["w_o"][p2]
    phi2, m2 = O.enhance(x, mq)
    assert torch.allclose(phi, phi2, atol=1e-13) and torch.allclose(m, m2, atol=1e-13)
    # zero head weights: phi = ReLU(b_phi) = 1 (the initialisation of Sec. 3.4), m = sigma(b_o)
    mz = dict(mp)
    mz["w_phi"] = torch.zeros(64, dtype=torch.float64)
    mz["w_o"] = torch.zeros(64, dtype=torch.float64)
    phi3, m3 = O.enhance(x, mz)
    assert float((phi3 - 1).abs().max()) == 0.0
    assert float((m3 - 1 / (1 + math.exp(-2.0))).abs().max()) < 1e-15


def test_mlp_f_256_128_64_matches_a_loop_over_neurons():
    """The appendix's MLP_f (ReLU layers of 256, 128, 64) against plain Python loops over
    the neurons of every layer for a few Gaussians (brute force, independent of the matrix
    products)."""
    mlp = mgs_data.make_mlp_f(21)
    mp = O.mlp_params(mlp)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(3, 22))
    phi, m = O.enhance(torch.tensor(x), mp)
    for g in range(3):
        h = [float(v) for v in x[g]]
        for k in (1, 2, 3):
            W, b = mlp[f"W{k}"].astype(np.float64), mlp[f"b{k}"].astype(np.float64)
            h = [max(0.0, sum(W[i][j] * h[j] for j in range(len(h))) + b[i]) for i in range(W.shape[0])]
        assert len(h) == 64
        zp = sum(float(mlp["w_phi"][i]) * h[i] for i in range(64)) + float(mlp["b_phi"])
        zo = sum(float(mlp["w_o"][i]) * h[i] for i in range(64)) + float(mlp["b_o"])
        assert abs(float(phi[g]) - max(0.0, zp)) < 1e-12
        assert abs(float(m[g]) - 1.0 / (1.0 + math.exp(-zo))) < 1e-12


def test_mlp_identity_layer_leaves_the_output_unchanged():
    """A third hidden layer that is the identity (on ReLU outputs, which are >= 0) gives the
    two-layer network's result: the layers are chained in order, each exactly once."""
    mp = _mlp64()
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.normal(size=(30, 22)))
    phi, m = O.enhance(x, mp)
    deep = dict(mp)
    deep["W3"] = torch.eye(64, dtype=torch.float64)
    deep["b3"] = torch.zeros(64, dtype=torch.float64)
    phi3, m3 = O.enhance(x, deep)
    assert torch.equal(phi, phi3) and torch.equal(m, m3)
    # ... and a non-identity third layer changes it
    deep["W3"] = torch.eye(64, dtype=torch.float64).roll(1, dims=0) * 0.5
    phi4, _ = O.enhance(x, deep)
    assert not torch.allclose(phi, phi4)


def test_bf16_rounding_is_round_to_nearest_even():
    v = torch.tensor([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 1 + 2 ** -8 + 2 ** -20, 3.0],
                     dtype=torch.float64)
    r = O.bf16_round(v)
    assert r.tolist() == [1.0, 1 + 2 ** -6, -1.0, 1 + 2 ** -7, 3.0]


def test_mlp_off_means_phi_one_m_one():
    sc, cam = _small(n=20)
    p = O.scene_params(sc)
    pr = O.project(p, cam)
    act = O.activate(p)
    _, d, _ = O.camera_space(p["mean"], cam)
    assert torch.allclose(pr["w"], O.depth_weight(torch.ones(20, dtype=torch.float64), d, act["s"]))
    assert torch.allclose(pr["o_eff"], act["o"])


# ---------------------------------------------------------------- gradients
def test_oracle_autograd_matches_central_differences():
    sc, cam = _small(n=12, seed=9, W=24, H=20)
    mlp = mgs_data.make_mlp(2)
    rng = np.random.default_rng(5)
    r = torch.tensor(rng.normal(size=(3, 20, 24)))
    bg = np.array([0.2, 0.5, 0.1])

    def loss(p, mp):
        act = O.activate(p)
        _, _, P = O.camera_space(p["mean"], cam)
        phi, m = O.enhance(O.mlp_features(P, act["s"], act["q"], p["sh"]), mp)
        pr = O.project(p, cam, phi, m)
        img, _ = O.render_oit(pr, cam, bg)
        return (img * r).sum(), pr

    p = O.scene_params(sc, requires_grad=True)
    mp = O.mlp_params(mlp, requires_grad=True)
    L, pr0 = loss(p, mp)
    L.backward()
    checked = 0
    rng2 = np.random.default_rng(1)
    for name in ("mean", "log_scale", "quat", "opacity_logit", "sh"):
        flat = p[name].detach().reshape(-1)
        g_ad = p[name].grad.reshape(-1)
        for idx in rng2.choice(flat.numel(), size=min(6, flat.numel()), replace=False):
            h = 1e-6 * max(1.0, abs(float(flat[idx])))
            vals = []
            for sgn in (1, -1):
                q = {k: v.detach().clone() for k, v in p.items()}
                q[name].view(-1)[idx] += sgn * h
                Lq, prq = loss(q, {k: v.detach() for k, v in mp.items()})
                vals.append((float(Lq), prq))
            # skip if the perturbation moved any pair across the alpha cut or a rect edge
            if any(not torch.equal(v[1]["rect"], pr0["rect"]) for v in vals):
                continue
            fd = (vals[0][0] - vals[1][0]) / (2 * h)
            assert abs(fd - float(g_ad[idx])) <= 1e-5 * (1 + abs(fd)), (name, idx, fd, float(g_ad[idx]))
            checked += 1
    for name in ("W2", "b1"):
        flat = mp[name].detach().reshape(-1)
        g_ad = mp[name].grad.reshape(-1)
        for idx in rng2.choice(flat.numel(), size=4, replace=False):
            h = 1e-6
            vals = []
            for sgn in (1, -1):
                mq = {k: v.detach().clone() for k, v in mp.items()}
                mq[name].view(-1)[idx] += sgn * h
                vals.append(float(loss({k: v.detach() for k, v in p.items()}, mq)[0]))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - float(g_ad[idx])) <= 1e-5 * (1 + abs(fd)), (name, idx)
            checked += 1
    assert checked >= 20


def test_bf16_rounding_passes_gradients_straight_through():
    x = torch.tensor([0.1234567, -3.3, 7.0], dtype=torch.float64, requires_grad=True)
    y = O.bf16_round(x)
    assert y.tolist() == O.bf16_round(x.detach()).tolist()
    (y * torch.tensor([0.3, -1.7, 2.5], dtype=torch.float64)).sum().backward()
    assert x.grad.tolist() == [0.3, -1.7, 2.5]          # not rounded to bfloat16


# --------------------------------------------------------------------------
# Vector-quantised attributes (Sec. 3.2): the decode is a lookup.
# --------------------------------------------------------------------------
def test_nvq_decode_hand_built_codebook():
    """Codeword value j of row b in codebook g is 1000 g + b + j / 8 (exact in float32), so
    every decoded attribute names its group, row and slot."""
    g_ = np.arange(5)[:, None, None]
    b_ = np.arange(1024)[None, :, None]
    j_ = np.arange(4)[None, None, :]
    cb = (1000.0 * g_ + b_ + j_ / 8.0).astype(np.float32)
    rng = np.random.default_rng(0)
    codes = rng.integers(0, 1024, size=(5, 300)).astype(np.uint16)
    mean = rng.normal(size=(3, 300)).astype(np.float32)
    sc = O.nvq.decode(codes, cb, mean)
    c = codes.astype(np.float64)
    for a in range(3):
        assert np.array_equal(sc["log_scale"][a], (c[0] + a / 8.0).astype(np.float32))
    assert np.array_equal(sc["quat"][0], (c[0] + 3 / 8.0).astype(np.float32))
    for a in range(3):
        assert np.array_equal(sc["quat"][1 + a], (1000 + c[1] + a / 8.0).astype(np.float32))
    assert np.array_equal(sc["opacity_logit"], (1000 + c[1] + 3 / 8.0).astype(np.float32))
    for k in range(12):
        g = 2 + k // 4
        assert np.array_equal(sc["sh"][k], (1000 * g + c[g] + (k % 4) / 8.0).astype(np.float32))
    assert np.array_equal(sc["mean"], mean)


def test_nvq_identity_codebook_reproduces_the_scene():
    """Codebooks holding a scene's own sub-vectors, with code = Gaussian index, decode back to
    the scene exactly (N <= 1024)."""
    scene = mgs_data.make_scene_uniform(700, 5)
    rows = np.concatenate([scene["log_scale"].T, scene["quat"].T, scene["opacity_logit"][:, None],
                           scene["sh"].T], axis=1)
    cb = np.zeros((5, 1024, 4), np.float32)
    for g in range(5):
        cb[g, :700] = rows[:, 4 * g:4 * g + 4]
    codes = np.tile(np.arange(700, dtype=np.uint16), (5, 1))
    sc = O.nvq.decode(codes, cb, scene["mean"])
    for k in ("mean", "log_scale", "quat", "opacity_logit", "sh"):
        assert np.array_equal(sc[k], scene[k]), k


def test_make_nvq_keeps_positions_and_draws_codewords_from_the_scene():
    scene = mgs_data.make_scene_uniform(5000, 6)
    q = mgs_data.make_nvq(scene, 7)
    assert q["codes"].dtype == np.uint16 and q["codes"].shape == (5, 5000) and q["codes"].max() < 1024
    assert q["codebooks"].shape == (5, 1024, 4) and np.array_equal(q["mean"], scene["mean"])
    rows = {tuple(r) for r in np.concatenate([scene["log_scale"].T, scene["quat"].T[:, :1]], axis=1)}
    assert all(tuple(r) in rows for r in q["codebooks"][0])
