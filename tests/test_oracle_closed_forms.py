"""More pins of the FP64 oracle: closed forms a wrong weight, clamp, stop rule, Jacobian
clamp, support rectangle, ambiguity set or per-tile depth order would fail.

Each expected value is written out here from the paper's formulas (Eq. 2 and Eq. 3 of
Sec. 3.1, Eq. 1 of Sec. 2, Eq. 11 of Appendix B) or from an enumeration that does not go
through the oracle's own code path; none of them comes from the HIP path.
"""
import math

import numpy as np
import pytest
import torch

import mgs_data
import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")

C0 = 1.0 / (2.0 * math.sqrt(math.pi))          # real SH, l = 0
F32 = lambda v: float(np.float32(v))            # scene inputs are stored as float32


def _gauss(mean, log_scale, logit, sh0=(0.0, 0.0, 0.0), quat=(1, 0, 0, 0)):
    sh = np.zeros((4, 3))
    sh[0] = sh0
    return dict(mean=np.asarray(mean, np.float32).reshape(3, 1),
                log_scale=np.asarray(log_scale, np.float32).reshape(3, 1),
                quat=np.asarray(quat, np.float32).reshape(4, 1),
                opacity_logit=np.asarray([logit], np.float32),
                sh=np.asarray(sh, np.float32).reshape(1, 12).T.copy())


def _cat(*gs):
    return {k: np.concatenate([g[k] for g in gs], axis=-1) for k in gs[0]}


def _sig(x):
    return 1.0 / (1.0 + math.exp(-x))


def _cam(W, H, f, z=4.0):
    """Camera at (0, 0, -z) looking down +z: R = I, t = (0, 0, z), principal point (W/2, H/2)."""
    return O.camera_tensors(mgs_data.look_at((0.0, 0.0, -z), width=W, height=H, f=f))


def _iso_on_axis(zw, ls, logit, sh0, f, z_cam=4.0):
    """Hand values of an isotropic Gaussian on the optical axis at world z = zw: depth,
    screen variance (f s / d)^2 + 0.3, opacity, SH0 colour and the Eq. 3 weight with phi = 1."""
    d = z_cam + F32(zw)
    s = math.exp(F32(ls))
    var = (f * s / d) ** 2 + 0.3
    o = _sig(F32(logit))
    c = np.maximum(0.0, 0.5 + C0 * np.array([F32(v) for v in sh0]))
    w = 1.0 + 1.0 / (d * d) + math.exp(s / d)       # phi^2 + phi / d^2 + exp(s_max / d), phi = 1
    return d, var, o, c, w


def _eq2(parts, bg, amin=1 / 255, amax=0.99):
    """Eq. 2 for one pixel from (a, c, w) of every Gaussian: skip a < amin, alpha = min(a, amax)."""
    num = np.zeros(3)
    den = 0.0
    T = 1.0
    for a, c, w in parts:
        if a < amin:
            continue
        al = min(a, amax)
        num += c * al * w
        den += al * w
        T *= 1.0 - al
    if den == 0.0:
        return np.asarray(bg, np.float64)
    return (1.0 - T) * num / den + T * np.asarray(bg, np.float64)


# ---------------------------------------------------------------- Eq. 2 with Eq. 3's weight
def test_two_cocentred_gaussians_weighted_average():
    """Two Gaussians on the axis at depths 2 and 7 with different colours and sizes: the
    image is Eq. 2's w-weighted average, w from Eq. 3 written out by hand."""
    W = H = 15                                   # odd: pixel (7, 7) is centred on the axis
    f = 15.0
    cam = _cam(W, H, f)
    g1 = dict(zw=-2.0, ls=-1.2, logit=0.4, sh0=(1.2, -0.8, 0.3))
    g2 = dict(zw=3.0, ls=-0.6, logit=1.1, sh0=(-0.9, 1.0, -1.2))
    sc = _cat(*(_gauss((0, 0, g["zw"]), (g["ls"],) * 3, g["logit"], g["sh0"]) for g in (g1, g2)))
    bg = np.array([0.15, 0.55, 0.35])
    img, aux = O.render_oit(O.project(O.scene_params(sc), cam), cam, bg)
    h1 = _iso_on_axis(g1["zw"], g1["ls"], g1["logit"], g1["sh0"], f)
    h2 = _iso_on_axis(g2["zw"], g2["ls"], g2["logit"], g2["sh0"], f)
    assert abs(h1[4] - h2[4]) > 0.2 and np.abs(h1[3] - h2[3]).min() > 0.2   # w and c differ
    checked = 0
    for (i, j) in ((7, 7), (6, 7), (9, 5), (3, 11), (12, 12), (0, 0)):
        r2 = (i - 7) ** 2 + (j - 7) ** 2
        parts = [(h[2] * math.exp(-0.5 * r2 / h[1]), h[3], h[4]) for h in (h1, h2)]
        ref = _eq2(parts, bg)
        assert np.abs(img[:, j, i].numpy() - ref).max() < 1e-12, (i, j)
        checked += all(a >= 1 / 255 for a, _, _ in parts)
    assert checked >= 3                          # several pixels see both Gaussians


def test_alpha_max_clamp_in_T_and_D():
    """Logit 8 puts the peak opacity at 0.99966 > alpha_max: at the centre pixel alpha = 0.99 in
    both the transmittance and the weighted sums (D is read back through aux)."""
    W = H = 15
    f = 15.0
    cam = _cam(W, H, f)
    ga = dict(zw=-1.0, ls=0.0, logit=8.0, sh0=(1.0, 0.2, -0.4))
    gb = dict(zw=1.0, ls=-0.8, logit=0.5, sh0=(-0.5, 0.7, 0.9))
    sc = _cat(*(_gauss((0, 0, g["zw"]), (g["ls"],) * 3, g["logit"], g["sh0"]) for g in (ga, gb)))
    bg = np.array([0.6, 0.1, 0.3])
    img, aux = O.render_oit(O.project(O.scene_params(sc), cam), cam, bg)
    ha = _iso_on_axis(ga["zw"], ga["ls"], ga["logit"], ga["sh0"], f)
    hb = _iso_on_axis(gb["zw"], gb["ls"], gb["logit"], gb["sh0"], f)
    assert ha[2] > 0.995
    # centre pixel: alpha_a = min(o_a, 0.99) = 0.99 exactly
    ab = hb[2]
    D_ref = 0.99 * ha[4] + ab * hb[4]
    T_ref = (1 - 0.99) * (1 - ab)
    assert abs(float(aux[3, 7, 7]) - D_ref) < 1e-12
    assert abs(float(aux[4, 7, 7]) - T_ref) < 1e-15
    ref = _eq2([(ha[2], ha[3], ha[4]), (ab, hb[3], hb[4])], bg)
    assert np.abs(img[:, 7, 7].numpy() - ref).max() < 1e-12
    # a single clamped Gaussian alone: C = 0.99 c + 0.01 bg
    sc1 = _gauss((0, 0, ga["zw"]), (ga["ls"],) * 3, ga["logit"], ga["sh0"])
    img1, aux1 = O.render_oit(O.project(O.scene_params(sc1), cam), cam, bg)
    assert np.abs(img1[:, 7, 7].numpy() - (0.99 * ha[3] + 0.01 * bg)).max() < 1e-13
    assert abs(float(aux1[4, 7, 7]) - 0.01) < 1e-15


# ---------------------------------------------------------------- Eq. 11 early stop
def test_sorted_early_stop_exact_value():
    """Five co-centred layers of alpha ~0.95 at depths 3 .. 5: the transmittance before the
    fourth is 0.05^3 = 1.25e-4 >= 1e-4 (composited), before the fifth 6.25e-6 (stopped).
    The value with no stop, or with one layer fewer, differs by more than 1e-7."""
    W = H = 9
    f = 9.0
    cam = _cam(W, H, f)
    logit = math.log(19.0)
    cols = [(1.4, -0.3, 0.2), (-0.6, 0.9, 0.1), (0.3, 0.3, -1.0), (0.8, -1.0, 0.6), (1.5, 1.5, 1.5)]
    zs = [-1.0, -0.5, 0.0, 0.5, 1.0]
    layers = [_gauss((0, 0, z), (1.0,) * 3, logit, c) for z, c in zip(zs, cols)]
    bg = np.array([0.9, 0.05, 0.4])
    ref_stop = ref_all = ref_short = None
    a = _sig(F32(logit))
    cs = [np.maximum(0.0, 0.5 + C0 * np.array([F32(v) for v in c])) for c in cols]

    def composite(k_live):
        out = np.zeros(3)
        T = 1.0
        for k in range(k_live):
            out += cs[k] * a * T
            T *= 1.0 - a
        return out + T * bg

    ref_stop, ref_all, ref_short = composite(4), composite(5), composite(3)
    assert np.abs(ref_stop - ref_all).max() > 1e-6 and np.abs(ref_stop - ref_short).max() > 1e-5
    for perm in ([0, 1, 2, 3, 4], [4, 2, 0, 3, 1]):      # list order does not matter
        pr = O.project(O.scene_params(_cat(*(layers[k] for k in perm))), cam)
        img = O.render_sorted(pr, cam, bg).numpy()
        assert np.abs(img[:, 4, 4] - ref_stop).max() < 1e-12


# ---------------------------------------------------------------- EWA frustum clamp
def test_ewa_jacobian_clamped_at_the_frustum_edge():
    """Isotropic Gaussians (s^2 I) seen by R = I: Sigma' = s^2 J J^T + 0.3 I with J taken at
    x/z, y/z clamped to +-1.3 (W/2)/fx, +-1.3 (H/2)/fy -- written out by hand.  W != H, so
    a limit taken from the wrong image side fails."""
    W, H, f, zc = 64, 32, 32.0, 4.0
    cam = _cam(W, H, f, zc)
    lim_x, lim_y = 1.3 * (W / 2) / f, 1.3 * (H / 2) / f         # 1.3 and 0.65
    ls = -1.5
    s2 = math.exp(F32(ls)) ** 2
    cases = [(2.0, 0.3), (1.0, 0.3), (0.2, -1.0), (-1.7, 0.9), (0.5, 0.5), (-3.0, -2.0)]
    sc = _cat(*(_gauss((rx * 5.0, ry * 5.0, 5.0 - zc), (ls,) * 3, 0.0) for rx, ry in cases))
    pr = O.project(O.scene_params(sc), cam)
    for g, (rx, ry) in enumerate(cases):
        xw, yw, zw = F32(rx * 5.0), F32(ry * 5.0), F32(5.0 - zc)
        d = zw + zc
        tx = min(max(xw / d, -lim_x), lim_x)
        ty = min(max(yw / d, -lim_y), lim_y)
        J = np.array([[f / d, 0.0, -f * tx / d], [0.0, f / d, -f * ty / d]])
        ref = s2 * J @ J.T + 0.3 * np.eye(2)
        assert np.abs(pr["cov2d"][g].numpy() - ref).max() < 1e-12 * (1 + np.abs(ref).max()), g
        # the mean itself is never clamped
        assert abs(float(pr["mean2d"][g, 0]) - (f * xw / d + W / 2)) < 1e-12
        assert abs(float(pr["mean2d"][g, 1]) - (f * yw / d + H / 2)) < 1e-12


# ---------------------------------------------------------------- rect tightness
def test_pixel_range_is_exactly_the_columns_and_rows_the_support_meets():
    """With tile = 1 the rect is the pixel range.  Enumerate every pixel column (row): it
    belongs to the range iff the line x = i + 1/2 (y = j + 1/2) meets the support
    {q <= 2 ln(o_eff / alpha_min)}.  Along the line q is a parabola in the free coordinate,
    whose minimum from the conic (A, B, C) is dx^2 (A - B^2 / C) (dy^2 (C - B^2 / A))."""
    W, H = 61, 47
    cam = O.camera_tensors(mgs_data.look_at((0.3, -0.2, -3.2), target=(0.05, 0.1, 0.0), width=W, height=H,
                                            f=55.0))
    sc = mgs_data.make_scene_uniform(80, seed=23, half=1.0, ls_mu=-2.3)
    pr = O.project(O.scene_params(sc), cam, tile=1)
    pr16 = O.project(O.scene_params(sc), cam, tile=16)
    seen = 0
    for g in range(80):
        if float(pr["depth"][g]) <= 0.2:
            continue
        o = float(pr["o_eff"][g])
        if o < 1 / 255:
            assert not bool(pr["visible"][g])
            continue
        k = 2.0 * math.log(o * 255.0)
        A, B, Cc = (float(v) for v in pr["conic"][g])
        mx, my = (float(v) for v in pr["mean2d"][g])
        qx = [(i + 0.5 - mx) ** 2 * (A - B * B / Cc) for i in range(W)]
        qy = [(j + 0.5 - my) ** 2 * (Cc - B * B / A) for j in range(H)]
        if any(abs(v - k) < 1e-9 * (1 + k) for v in qx + qy):
            continue                                 # a line grazes the support: undecidable here
        cols = [i for i in range(W) if qx[i] <= k]
        rows = [j for j in range(H) if qy[j] <= k]
        if not cols or not rows:
            assert not bool(pr["visible"][g]) and int(pr["n_tiles"][g]) == 0
            continue
        seen += 1
        assert bool(pr["visible"][g])
        assert pr["rect"][g].tolist() == [cols[0], rows[0], cols[-1], rows[-1]], g
        assert int(pr["n_tiles"][g]) == len(cols) * len(rows)
        assert pr16["rect"][g].tolist() == [cols[0] // 16, rows[0] // 16, cols[-1] // 16, rows[-1] // 16]
    assert seen >= 25


# ---------------------------------------------------------------- ambiguity set
def _handmade(cam, g):
    """A projected-Gaussian table written directly: every Gaussian peaks exactly on a pixel
    centre (conic 40 I: far pixels see nothing)."""
    n = len(g)
    t = lambda v: torch.tensor(v, dtype=torch.float64)
    return dict(mean2d=t([x["m"] for x in g]), conic=t([[40.0, 0.0, 40.0]] * n), o_eff=t([x["o"] for x in g]),
                color=t([x["c"] for x in g]), w=t([x["w"] for x in g]), depth=t([x.get("d", 1.0) for x in g]),
                depth_mag=t([abs(x.get("d", 1.0)) for x in g]), visible=torch.ones(n, dtype=torch.bool))


def test_ambiguity_variants_are_exactly_the_admissible_images():
    """Pixel 0 sees a clear contributor, one pair at alpha_min (1 + 5e-5) (nominally in) and one
    at alpha_min (1 - 5e-5) (nominally out): the four variants are the images of the four
    include/exclude choices.  Pixel 2 has three ambiguous pairs and is flagged."""
    amin = 1 / 255
    cam = dict(W=3, H=1)
    gs = [dict(m=[0.5, 0.5], o=0.5, c=[0.9, 0.2, 0.1], w=1.7),
          dict(m=[0.5, 0.5], o=amin * (1 + 5e-5), c=[0.0, 1.0, 0.3], w=2.9),
          dict(m=[0.5, 0.5], o=amin * (1 - 5e-5), c=[0.4, 0.0, 1.0], w=0.6),
          dict(m=[1.5, 0.5], o=0.3, c=[0.2, 0.2, 0.8], w=1.1)]
    gs += [dict(m=[2.5, 0.5], o=amin * (1 + s), c=[0.1 * k, 0.5, 0.2], w=1.0 + k)
           for k, s in enumerate((3e-5, -2e-5, 6e-5))]
    pr = _handmade(cam, gs)
    bg = np.array([0.25, 0.5, 0.75])
    for w_bg in (None, 0.8):
        img, aux, V, flagged = O.render_oit(pr, cam, bg, variants=True, w_bg=w_bg)
        assert flagged == 1

        def pix0(members):
            num, den, T = np.zeros(3), 0.0, 1.0
            for k in members:
                num += np.array(gs[k]["c"]) * gs[k]["o"] * gs[k]["w"]
                den += gs[k]["o"] * gs[k]["w"]
                T *= 1 - gs[k]["o"]
            if w_bg is not None:
                return (num + w_bg * bg) / (den + w_bg)
            return (1 - T) * num / den + T * bg

        expect = [pix0(m) for m in ([0, 1], [0], [0, 1, 2], [0, 2])]
        got = [V[v, :, 0, 0].numpy() for v in range(4)]
        assert np.abs(got[0] - expect[0]).max() < 1e-13          # variant 0 is the nominal image
        assert np.abs(img[:, 0, 0].numpy() - expect[0]).max() < 1e-13
        for e in expect:                                        # the sets are equal
            assert min(np.abs(gv - e).max() for gv in got) < 1e-13
        for gv in got:
            assert min(np.abs(gv - e).max() for e in expect) < 1e-13
        # pixel 1 has no ambiguous pair: every variant is its one image
        assert float((V[:, :, 0, 1] - img[None, :, 0, 1]).abs().max()) < 1e-15


# ---------------------------------------------------------------- Eq. 1 (SortFreeGS composite)
def test_sortfree_weight_and_composite_closed_form():
    """Eq. 1: C = (c_bg w_bg + sum c a w) / (w_bg + sum a w), w = exp(-sigma d^beta), for two
    co-centred Gaussians; w_bg -> large gives the background; no Gaussian gives c_bg."""
    W = H = 15
    f = 15.0
    cam = _cam(W, H, f)
    g1 = dict(zw=-1.0, ls=-1.0, logit=0.8, sh0=(1.0, -0.5, 0.2))
    g2 = dict(zw=1.5, ls=-0.7, logit=1.6, sh0=(-0.7, 0.9, 0.4))
    sc = _cat(*(_gauss((0, 0, g["zw"]), (g["ls"],) * 3, g["logit"], g["sh0"]) for g in (g1, g2)))
    sigma = np.array([0.35, 0.12])
    beta = np.array([1.3, 0.7])
    p = O.scene_params(sc)
    sf = (torch.tensor(sigma), torch.tensor(beta))
    pr = O.project(p, cam, weight_mode=O.WEIGHT_SORTFREE, sortfree=sf)
    h = [_iso_on_axis(g["zw"], g["ls"], g["logit"], g["sh0"], f) for g in (g1, g2)]
    wsf = [math.exp(-sigma[k] * h[k][0] ** beta[k]) for k in range(2)]
    assert np.allclose(pr["w"].numpy(), wsf, rtol=1e-14, atol=0)
    bg = np.array([0.3, 0.8, 0.1])
    for w_bg in (0.0, 0.45, 2.0):
        img, _ = O.render_oit(pr, cam, bg, w_bg=w_bg)
        for (i, j) in ((7, 7), (5, 8), (10, 3), (0, 14)):
            r2 = (i - 7) ** 2 + (j - 7) ** 2
            num, den = w_bg * bg, w_bg
            for k in range(2):
                a = h[k][2] * math.exp(-0.5 * r2 / h[k][1])
                if a >= 1 / 255:
                    al = min(a, 0.99)
                    num = num + h[k][3] * al * wsf[k]
                    den += al * wsf[k]
            ref = num / den if den > 0 else bg
            assert np.abs(img[:, j, i].numpy() - ref).max() < 1e-12, (w_bg, i, j)
    big, _ = O.render_oit(pr, cam, bg, w_bg=1e12)
    assert float((big - torch.tensor(bg)[:, None, None]).abs().max()) < 1e-10
    # sigma = 0: w = 1, so the composite is the plain alpha-weighted average
    pr0 = O.project(p, cam, weight_mode=O.WEIGHT_SORTFREE, sortfree=(torch.zeros(2), torch.tensor(beta)))
    assert torch.equal(pr0["w"], torch.ones(2, dtype=torch.float64))
    with pytest.raises(ValueError):
        O.project(p, cam, weight_mode=O.WEIGHT_SORTFREE)


def test_sortfree_composite_ignores_order_and_transmittance():
    """Eq. 1 has no T: duplicating every Gaussian (which squares T) and scaling w_bg by two
    leaves the image unchanged; permuting the Gaussians leaves it unchanged."""
    sc = mgs_data.make_scene_uniform(40, seed=9, half=0.9, ls_mu=-2.6)
    cam = mgs_data.look_at((0.2, -0.1, -3.5), width=36, height=30, f=40.0)
    rng = np.random.default_rng(4)
    sigma, beta = rng.uniform(0.05, 0.5, 40), rng.uniform(0.5, 2.0, 40)
    bg = np.array([0.2, 0.4, 0.6])
    img, _, _ = O.render(sc, cam, bg=bg, weight_mode=O.WEIGHT_SORTFREE, sortfree=(sigma, beta), w_bg=0.3)
    dup = {k: np.concatenate([v, v], axis=-1) for k, v in sc.items()}
    img2, _, _ = O.render(dup, cam, bg=bg, weight_mode=O.WEIGHT_SORTFREE,
                          sortfree=(np.tile(sigma, 2), np.tile(beta, 2)), w_bg=0.6)
    assert float((img - img2).abs().max()) < 1e-13
    perm = rng.permutation(40)
    scp = {k: v[..., perm] for k, v in sc.items()}
    img3, _, _ = O.render(scp, cam, bg=bg, weight_mode=O.WEIGHT_SORTFREE, sortfree=(sigma[perm], beta[perm]),
                          w_bg=0.3)
    assert float((img - img3).abs().max()) < 1e-13
    assert float(img.std()) > 1e-3


# ---------------------------------------------------------------- per-tile depth order
def test_bin_lists_sorted_equals_bruteforce_depth_order():
    """Each tile's list = the Gaussians whose rect covers it (O(N T) enumeration), ordered by
    (depth, index) with Python's tuple sort; exact depth ties are included."""
    rng = np.random.default_rng(31)
    tx, ty, n = 6, 5, 250
    x0 = rng.integers(0, tx, n)
    y0 = rng.integers(0, ty, n)
    x1 = np.minimum(tx - 1, x0 + rng.integers(0, 3, n))
    y1 = np.minimum(ty - 1, y0 + rng.integers(0, 3, n))
    rect = np.stack([x0, y0, x1, y1], 1)
    nt = (x1 - x0 + 1) * (y1 - y0 + 1)
    nt[rng.random(n) < 0.15] = 0
    rect[nt == 0] = 0
    depth = rng.choice(np.linspace(0.5, 9.0, 40), n)          # many exact ties
    offs, gids = O.bin_lists_sorted(rect, nt, depth, tx, ty)
    ref_offs, ref = [0], []
    for t in range(tx * ty):
        cx, cy = t % tx, t // tx
        members = [g for g in range(n) if nt[g] > 0 and x0[g] <= cx <= x1[g] and y0[g] <= cy <= y1[g]]
        ref += sorted(members, key=lambda g: (depth[g], g))
        ref_offs.append(len(ref))
    assert offs.tolist() == ref_offs and gids.tolist() == ref


def test_sorted_flags_mark_exactly_the_fragile_pixels():
    """render_sorted's flags: a depth tie below the float32 key's error bound (8 x 2^-24 x the
    depth's magnitude per key), a transmittance within 0.1% of the stop value, or an
    ambiguous alpha cut each flag their pixel; a clean pixel, a gap just above the bound and a
    tie behind the stop are not flagged."""
    amin = 1 / 255
    cam = dict(W=6, H=1)
    a_stop = 1.0 - 1e-4 * (1 + 2e-4)           # T before the next pair = 1e-4 (1 + 2e-4)
    bound = 8 * 2.0 ** -24 * (2.0 + 2.0)        # tie bound of two keys at depth 2
    gs = [dict(m=[0.5, 0.5], o=0.6, c=[1, 0, 0], w=1.0, d=2.0),              # pixel 0: clean
          dict(m=[0.5, 0.5], o=0.3, c=[0, 1, 0], w=1.0, d=3.0),
          dict(m=[1.5, 0.5], o=0.6, c=[1, 0, 0], w=1.0, d=2.0),              # pixel 1: depth tie
          dict(m=[1.5, 0.5], o=0.3, c=[0, 1, 0], w=1.0, d=2.0 + 0.5 * bound),
          dict(m=[2.5, 0.5], o=a_stop, c=[1, 0, 0], w=1.0, d=2.0),           # pixel 2: near stop
          dict(m=[2.5, 0.5], o=0.5, c=[0, 0, 1], w=1.0, d=4.0),
          dict(m=[3.5, 0.5], o=amin * (1 + 1e-5), c=[1, 1, 0], w=1.0, d=2.0),  # pixel 3: ambiguous
          dict(m=[3.5, 0.5], o=0.2, c=[0, 1, 1], w=1.0, d=3.0),
          dict(m=[4.5, 0.5], o=0.6, c=[1, 0, 0], w=1.0, d=2.0),              # pixel 4: gap > bound
          dict(m=[4.5, 0.5], o=0.3, c=[0, 1, 0], w=1.0, d=2.0 + 1.5 * bound),
          dict(m=[5.5, 0.5], o=0.999, c=[1, 0, 0], w=1.0, d=1.0),            # pixel 5: stop, then a tie
          dict(m=[5.5, 0.5], o=0.99, c=[0, 1, 0], w=1.0, d=1.5),
          dict(m=[5.5, 0.5], o=0.5, c=[0, 0, 1], w=1.0, d=2.0),
          dict(m=[5.5, 0.5], o=0.5, c=[1, 1, 1], w=1.0, d=2.0)]
    pr = _handmade(cam, gs)
    img, flags = O.render_sorted(pr, cam, np.zeros(3), alpha_max=0.9999, return_flags=True)
    assert flags[0].tolist() == [False, True, True, True, False, False]
    # the clean pixel's value: front-to-back by hand
    ref0 = 0.6 * np.array([1, 0, 0]) + 0.4 * 0.3 * np.array([0, 1, 0])
    assert np.abs(img[:, 0, 0].numpy() - ref0).max() < 1e-15
    # pixel 5 stops after two layers (T = 1e-5 < 1e-4)
    ref5 = 0.999 * np.array([1, 0, 0]) + 0.001 * 0.99 * np.array([0, 1, 0])
    assert np.abs(img[:, 0, 5].numpy() - ref5).max() < 1e-15


def test_sorted_binned_equals_bruteforce():
    """The per-tile sorted mode (each tile's list in (depth, index) order) gives the brute-force
    image and flags: a Gaussian outside a tile's list never reaches alpha_min there."""
    sc = mgs_data.make_scene_uniform(150, seed=17, half=0.9, ls_mu=-2.5)
    cam = O.camera_tensors(mgs_data.look_at((0.2, 0.1, -3.3), width=57, height=41, f=50.0))
    pr = O.project(O.scene_params(sc), cam)
    bg = np.array([0.3, 0.2, 0.6])
    a, fa = O.render_sorted(pr, cam, bg, return_flags=True)
    b, fb = O.render_sorted(pr, cam, bg, return_flags=True, mode="binned")
    assert float((a - b).abs().max()) < 1e-13 and torch.equal(fa, fb)
    assert float(a.std()) > 1e-3


def test_ambiguity_band_widens_with_the_screen_position_error():
    """A pair 6e-4 (in ln) below alpha_min, 0.1 px from its Gaussian's mean with conic 40 I:
    ln a moves by |A dx|_1 = 4 per pixel of mean error, so a position error bound of 2e-4 px
    makes it ambiguous (4 x 2e-4 + 1e-4 > 6e-4) and one of 1e-4 px does not."""
    amin = 1 / 255
    cam = dict(W=1, H=1)
    q = 40.0 * 0.1 ** 2
    o = amin * math.exp(-6e-4) * math.exp(0.5 * q)
    gs = [dict(m=[0.5, 0.5], o=0.4, c=[0.9, 0.1, 0.2], w=1.3),
          dict(m=[0.5, 0.5], o=o, c=[0.1, 0.8, 0.7], w=2.1)]
    bg = np.array([0.2, 0.2, 0.2])
    out_img = 0.4 * np.array([0.9, 0.1, 0.2]) + 0.6 * bg          # only the clear contributor
    a2 = amin * math.exp(-6e-4)
    num = 0.4 * 1.3 * np.array([0.9, 0.1, 0.2]) + a2 * 2.1 * np.array([0.1, 0.8, 0.7])
    T = 0.6 * (1 - a2)
    in_img = (1 - T) * num / (0.4 * 1.3 + a2 * 2.1) + T * bg
    for axis, pos, ambiguous in ((0, 2e-4, True), (0, 1e-4, False), (0, 0.0, False), (1, 2e-4, True),
                                 (1, 1e-4, False)):
        pr = _handmade(cam, gs)
        pr["mean2d"][1] = torch.tensor([0.5, 0.5], dtype=torch.float64)
        pr["mean2d"][1, axis] = 0.6                         # offset along x, then along y
        pr["pos_err"] = torch.tensor([0.0, pos], dtype=torch.float64)
        img, _, V, flagged = O.render_oit(pr, cam, bg, variants=True)
        assert np.abs(img[:, 0, 0].numpy() - out_img).max() < 1e-13
        got = [V[v, :, 0, 0].numpy() for v in range(4)]
        has_in = min(np.abs(gv - in_img).max() for gv in got) < 1e-13
        assert has_in == ambiguous, (axis, pos)
        _, flags = O.render_sorted(pr, cam, bg, return_flags=True)
        assert bool(flags[0, 0]) == ambiguous


def test_screen_position_error_bound_closed_form():
    """pos_err = POS_ULPS 2^-24 max over the axes of f (|R_row| . |mu| + |t_row|) / d + |c|,
    written out for an identity-rotation camera at (0, 0, -4)."""
    W, H, f = 64, 48, 50.0
    cam = _cam(W, H, f)
    pts = [(0.3, -0.2, 0.5), (-1.1, 0.4, -0.7), (0.0, 0.0, 2.0)]
    sc = _cat(*(_gauss(p, (-2.0,) * 3, 0.0) for p in pts))
    pr = O.project(O.scene_params(sc), cam)
    for g, (x, y, z) in enumerate(pts):
        x, y, z = F32(x), F32(y), F32(z)
        d = z + 4.0
        ref = 4.0 * 2.0 ** -24 * max(f * abs(x) / d + W / 2, f * abs(y) / d + H / 2)
        assert abs(float(pr["pos_err"][g]) - ref) < 1e-15 * (1 + ref), g


def test_ambiguous_gaussians_marks_pairs_at_either_cut():
    """A Gaussian with a pixel in the alpha_min band, one with a pixel in the alpha_max band and
    clear ones (peaks well inside, supports away from the cut at every pixel centre)."""
    amin, amax = 1 / 255, 0.99
    cam = dict(W=4, H=1)
    gs = [dict(m=[0.5, 0.5], o=0.5, c=[1, 0, 0], w=1.0),
          dict(m=[1.5, 0.5], o=amin * (1 + 3e-5), c=[0, 1, 0], w=1.0),
          dict(m=[2.5, 0.5], o=amax * (1 - 2e-5), c=[0, 0, 1], w=1.0),
          dict(m=[3.5, 0.5], o=0.97, c=[1, 1, 0], w=1.0)]
    pr = _handmade(cam, gs)
    pr.update(rect=torch.tensor([[0, 0, 0, 0]] * 4), n_tiles=torch.ones(4, dtype=torch.int64), tiles_x=1,
              tiles_y=1, tile=16)
    assert O.ambiguous_gaussians(pr, cam).tolist() == [False, True, True, False]
