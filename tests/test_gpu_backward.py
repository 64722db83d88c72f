"""Backward pass (mgs_render_backward via torch.autograd) against the oracle's FP64
autograd gradient and against finite differences of the GPU forward.

Bar: per parameter tensor, and per MLP layer (W1, b1, W2, b2, w_phi, b_phi, w_o, b_o each on
its own), ||g - g*||_2 / ||g*||_2 <= 1e-3 against the oracle; elementwise, every entry with
|g*| > 1e-3 max|g*| of its tensor within 1e-3 |g*| (plus 1e-6 max|g*| for rounding of
cancelling sums; 1e-5 max|g*| on dense scenes with the MLP, where the few Gaussians whose bf16
roundings flipped change the pixel sums their neighbours' gradients read).  The MLP's gradient
is taken straight through the forward's bfloat16 roundings on both sides (the oracle runs its
BF16-emulation forward).
"""
import numpy as np
import pytest
import torch

import mgs_data
import oracle as O
from gpu_helpers import oracle_project, say

pytestmark = pytest.mark.gpu

KEYS = ("mean", "log_scale", "quat", "opacity_logit", "sh")
REL = 1e-3


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11531_amd as M
    import paper_2603_11531_amd.autograd  # noqa: F401
    M._lib.lib()
    return M


def _flat_mlp(M, mlp):
    flat = np.zeros(M._lib.MGS_MLP_PARAMS, np.float32)
    for name, off, shape in M._lib.MLP_LAYOUT:
        v = np.asarray(mlp[name], np.float32).reshape(-1)
        flat[off:off + v.size] = v
    return flat


def gpu_grads(M, scene, cam, mlp, r, bg):
    from paper_2603_11531_amd.autograd import render
    params = {k: torch.tensor(np.ascontiguousarray(scene[k]), device="cuda", requires_grad=True) for k in KEYS}
    mp = torch.tensor(_flat_mlp(M, mlp), device="cuda", requires_grad=True) if mlp is not None else None
    img = render(params, cam, mp, bg)
    L = (img * torch.as_tensor(r, dtype=torch.float32, device="cuda")).sum()
    L.backward()
    torch.cuda.synchronize()
    out = {k: params[k].grad.double().cpu().numpy() for k in KEYS}
    if mp is not None:
        out["mlp"] = mp.grad.double().cpu().numpy()
    return out, img.detach().double().cpu()


HEADS = ("b_phi", "b_o")


def oracle_grads(M, scene, cam, mlp, r, bg, bf16=True, mode="brute"):
    """The oracle's FP64 gradients in the mgs.h layout.  The head biases b_phi and b_o are fed
    as one leaf per Gaussian, so their gradient is the sum of per-Gaussian terms t_i and
    out["abs_terms"][name] = sum |t_i| (the scale of the float32 error of that sum)."""
    camt = O.camera_tensors(cam)
    p = O.scene_params(scene, requires_grad=True)
    mp = O.mlp_params(mlp, requires_grad=True) if mlp is not None else None
    n = scene["mean"].shape[1]
    if mp is not None:
        for name in HEADS:
            mp[name] = mp[name].detach().expand(n).clone().requires_grad_(True)
    phi = m = None
    if mp is not None:
        act = O.activate(p)
        _, _, P = O.camera_space(p["mean"], camt)
        phi, m = O.enhance(O.mlp_features(P, act["s"], act["q"], p["sh"]), mp, bf16=bf16)
    pr = O.project(p, camt, phi, m)
    img, _ = O.render_oit(pr, camt, np.asarray(bg), mode=mode)
    (img * torch.as_tensor(r, dtype=torch.float64)).sum().backward()
    n = scene["mean"].shape[1]
    out = {"mean": p["mean"].grad.numpy().T, "log_scale": p["log_scale"].grad.numpy().T,
           "quat": p["quat"].grad.numpy().T, "opacity_logit": p["opacity_logit"].grad.numpy(),
           "sh": p["sh"].grad.numpy().reshape(n, 12).T}
    if mp is not None:
        flat = np.zeros(M._lib.MGS_MLP_PARAMS)
        for name, off, shape in M._lib.MLP_LAYOUT:
            v = mp[name].grad.numpy().reshape(-1)
            if name in HEADS:
                v = np.array([v.sum()])
            flat[off:off + v.size] = v
        out["mlp"] = flat
        out["abs_terms"] = {name: float(mp[name].grad.abs().sum()) for name in HEADS}
    return out, img.detach()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _parts(M, g):
    """Gradient tensors to check one by one: the five attribute tensors and each MLP layer."""
    out = {k: g[k] for k in KEYS}
    if "mlp" in g:
        for name, off, shape in M._lib.MLP_LAYOUT:
            sz = int(np.prod(shape)) if shape else 1
            out["mlp." + name] = g["mlp"][off:off + sz]
    return out


def mlp_flipped(M, scene, cam, mlp):
    """Gaussians whose float32 MLP outputs (phi, m) differ from the oracle's BF16 emulation by more
    than float32 rounding: a bf16 rounding of an input or hidden value fell the other way, so
    their forward, and with it their gradient, differs from the emulation's."""
    ds, dm = M.DeviceScene(scene), M.DeviceMLP(mlp)
    R = M.Renderer(ds.n, cam.width, cam.height)
    R.enhance(ds, M._lib.make_camera(cam), dm)
    torch.cuda.synchronize()
    camt = O.camera_tensors(cam)
    p = O.scene_params(scene)
    with torch.no_grad():
        act = O.activate(p)
        _, _, P = O.camera_space(p["mean"], camt)
        phi, m = O.enhance(O.mlp_features(P, act["s"], act["q"], p["sh"]), O.mlp_params(mlp), bf16=True)
    dphi = (R.phi.double().cpu() - phi).abs().numpy()
    dm_ = (R.omod.double().cpu() - m).abs().numpy()
    return (dphi > 1e-5 * (1 + np.abs(phi.numpy()))) | (dm_ > 1e-6)


def _check(M, g, go, skip=None, atol=1e-6, mlp_elementwise=True):
    """The bar of this module for every tensor and MLP layer; prints each figure.  ``skip``: a
    mask of Gaussians left out of the elementwise bar (their forward differs, see mlp_flipped);
    the L2 bar covers every entry.  ``mlp_elementwise=False`` keeps the MLP layers to the L2 bar:
    each weight-gradient entry sums over every Gaussian, so a skipped Gaussian's term cannot be
    left out of it."""
    a, b = _parts(M, g), _parts(M, go)
    terms = go.get("abs_terms", {})
    worst = {}
    for k in b:
        e = _rel(a[k], b[k])
        if k[4:] in terms:
            # a head bias's gradient sums one term per Gaussian, and Eq. 2's invariance to a common
            # scale of w makes the phi head's terms cancel (sum |t_i| / |sum t_i| reaches 1e6 on
            # dense scenes): its bar is relative to sum |t_i| as well
            tol = REL * abs(float(b[k][0])) + 1e-6 * terms[k[4:]]
            d0 = abs(float(a[k][0] - b[k][0]))
            say(f"  {k}: |g - g*| {d0:.3e}, |g*| {abs(float(b[k][0])):.3e}, sum |t_i| {terms[k[4:]]:.3e}, "
                f"bar {tol:.3e}")
            assert d0 <= tol, (k, d0, tol)
            worst[k] = e
            continue
        gm = float(np.abs(b[k]).max())
        big = np.abs(b[k]) > 1e-3 * gm
        if skip is not None and not k.startswith("mlp."):
            big &= ~np.broadcast_to(skip, b[k].shape)
        d = np.abs(a[k] - b[k])
        over = (d > 1e-3 * np.abs(b[k]) + atol * gm) & big
        rel_e = np.where(big, d / np.maximum(np.abs(b[k]), 1e-300), 0.0)
        say(f"  {k}: rel L2 {e:.2e}, elementwise worst {float(rel_e.max()):.2e} over bar {int(over.sum())} of "
            f"{int(big.sum())}")
        for flat in np.argsort(rel_e.reshape(-1))[::-1][:3] if over.any() else []:
            ix = np.unravel_index(flat, b[k].shape)
            say(f"    entry {tuple(int(v) for v in ix)}: |g*|/max {abs(b[k][ix]) / gm:.2e} "
                f"|g-g*|/max {d[ix] / gm:.2e} rel {rel_e[ix]:.2e}")
        assert e <= REL, (k, e)
        if mlp_elementwise or not k.startswith("mlp."):
            assert int(over.sum()) == 0, (k, int(over.sum()))
        worst[k] = e
    return worst


@pytest.mark.parametrize("with_mlp", [False, True])
def test_grads_match_oracle_tiny(M, with_mlp):
    say(f"test_grads_match_oracle_tiny mlp={with_mlp}")
    scene = mgs_data.make_scene_uniform(50, 21, half=0.8, ls_mu=-2.4)
    cam = mgs_data.look_at((0.0, 0.0, -4.0), width=32, height=32, f=32.0)
    mlp = mgs_data.make_mlp(22) if with_mlp else None
    rng = np.random.default_rng(3)
    r = rng.normal(size=(3, 32, 32))
    bg = (0.2, 0.4, 0.1)
    g, img = gpu_grads(M, scene, cam, mlp, r, bg)
    go, imgo = oracle_grads(M, scene, cam, mlp, r, bg)
    _check(M, g, go)


@pytest.mark.parametrize("with_mlp", [False, True])
def test_grads_match_oracle_small_workload(M, with_mlp):
    say(f"test_grads_match_oracle_small_workload mlp={with_mlp}")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    mlp = mgs_data.make_mlp(1) if with_mlp else None
    rng = np.random.default_rng(4)
    r = rng.normal(size=(3, 128, 128))
    bg = (0.0, 0.0, 0.0)
    g, _ = gpu_grads(M, scene, cams[0], mlp, r, bg)
    go, _ = oracle_grads(M, scene, cams[0], mlp, r, bg)
    _check(M, g, go)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("with_mlp", [False, True])
def test_grads_match_oracle_dense_tiles(M, with_mlp):
    """40,000 Gaussians filling a 96x96 view: every tile list holds 1,800-3,500 Gaussians (the
    training workload's density), so the backward walks many 256-Gaussian chunks per tile."""
    say(f"test_grads_match_oracle_dense_tiles mlp={with_mlp}")
    scene = mgs_data.make_scene_uniform(40000, 31, half=2.2, ls_mu=-2.5)
    cam = mgs_data.look_at((0.1, -0.1, -4.0), width=96, height=96, f=96.0)
    mlp = mgs_data.make_mlp(32) if with_mlp else None
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, cam.width, cam.height)
    R.render(ds, cam)
    offs, _ = R.lists()
    lens = (offs[1:] - offs[:-1])
    say(f"  tile lists: min {int(lens.min())} max {int(lens.max())}")
    assert int(lens.min()) > 1000
    rng = np.random.default_rng(6)
    r = rng.normal(size=(3, 96, 96))
    bg = (0.1, 0.3, 0.2)
    g, _ = gpu_grads(M, scene, cam, mlp, r, bg)
    go, _ = oracle_grads(M, scene, cam, mlp, r, bg, mode="binned")
    # A Gaussian with a pixel pair at the alpha_min cut (or the alpha_max clamp) that float32
    # may place on either side has two admissible gradients (the pair's term in or out); with
    # the MLP, one whose bf16 roundings flipped has a different forward.  Both are left out of
    # the elementwise bar (the L2 bar covers them).
    pr, camt = oracle_project(scene, cam, mlp=mlp, bf16=True)
    skip = O.ambiguous_gaussians(pr, camt).numpy()
    say(f"  Gaussians with a pair at a cut: {int(skip.sum())} of {skip.size}")
    if with_mlp:
        fl = mlp_flipped(M, scene, cam, mlp)
        say(f"  Gaussians with a flipped bf16 rounding: {int(fl.sum())}")
        skip = skip | fl
    _check(M, g, go, skip, atol=1e-5 if with_mlp else 1e-6, mlp_elementwise=False)


def test_grads_match_finite_differences_of_gpu_forward(M):
    """Central differences of the GPU forward (float32, h = 1e-3) on the 50-Gaussian 32x32 scene.

    With the MLP off the forward is smooth in every attribute; with the MLP on, only the
    two head biases enter after the bfloat16 roundings, so they are the MLP parameters
    a finite difference can probe (the rest is checked against the oracle above).
    """
    say("test_grads_match_finite_differences_of_gpu_forward")
    scene = mgs_data.make_scene_uniform(50, 21, half=0.8, ls_mu=-2.4)
    cam = mgs_data.look_at((0.0, 0.0, -4.0), width=32, height=32, f=32.0)
    mlp = mgs_data.make_mlp(22)
    rng = np.random.default_rng(3)
    r = rng.normal(size=(3, 32, 32))
    bg = (0.2, 0.4, 0.1)
    rt = torch.as_tensor(r, dtype=torch.float64)

    def loss(sc, flat):
        ds = M.DeviceScene(sc)
        R = M.Renderer(ds.n, 32, 32)
        dm = M.DeviceMLP(M.DeviceMLP.unflatten(flat)) if flat is not None else None
        img = R.render(ds, cam, dm, bg=bg).double().cpu()
        return float((img * rt).sum()), R.decoded()["rect"].copy()

    checked, bad = 0, []
    pick = np.random.default_rng(9)
    g, _ = gpu_grads(M, scene, cam, None, r, bg)
    _, rect0 = loss(scene, None)
    for k in ("mean", "log_scale", "opacity_logit", "sh", "quat"):
        arr = scene[k]
        for idx in pick.choice(arr.size, size=6, replace=False):
            h = 1e-3
            vals = []
            for sgn in (1, -1):
                sc = {kk: v.copy() for kk, v in scene.items()}
                sc[k].reshape(-1)[idx] += sgn * h
                vals.append(loss(sc, None))
            if any(not np.array_equal(v[1], rect0) for v in vals):
                continue
            fd = (vals[0][0] - vals[1][0]) / (2 * h)
            an = float(g[k].reshape(-1)[idx])
            scale = max(abs(fd), abs(an), 0.05 * float(np.abs(g[k]).max()), 1e-3)
            checked += 1
            if abs(fd - an) > 3e-2 * scale:
                bad.append((k, int(idx), fd, an))
    # MLP head biases.  A bias moves every pixel a little, and with a random weighting r the
    # loss change at h = 1e-3 is only ~10 float32 ulps of the loss, so the difference is
    # dominated by the forward's rounding.  The weighting is therefore aligned with the
    # image change, r_k = sign(C(b + H) - C(b - H)) at a wide H, which raises the signal
    # about sqrt(pixels)-fold at the same noise; the analytic gradient uses the same r_k.
    flat = _flat_mlp(M, mlp)

    def image(f):
        ds = M.DeviceScene(scene)
        R = M.Renderer(ds.n, 32, 32)
        return R.render(ds, cam, M.DeviceMLP(M.DeviceMLP.unflatten(f)), bg=bg).double().cpu()

    for off in (M._lib.MLP_LAYOUT[5][1], M._lib.MLP_LAYOUT[7][1]):      # b_phi, b_o
        wide = []
        for sgn in (1, -1):
            f2 = flat.copy()
            f2[off] += sgn * 3e-2
            wide.append(image(f2))
        rk = torch.sign(wide[0] - wide[1]).numpy()
        rkt = torch.as_tensor(rk)
        gm, _ = gpu_grads(M, scene, cam, mlp, rk, bg)
        h = 1e-3
        vals = []
        for sgn in (1, -1):
            f2 = flat.copy()
            f2[off] += sgn * h
            vals.append(float((image(f2) * rkt).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(gm["mlp"][off])
        checked += 1
        if abs(fd - an) > 3e-2 * max(abs(fd), abs(an), 1e-3):
            bad.append(("mlp", off, fd, an))
    say(f"  checked {checked}, mismatches {bad}")
    assert checked >= 15 and len(bad) <= 1, bad


def test_backward_is_bit_reproducible(M):
    say("test_backward_is_bit_reproducible")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    mlp = mgs_data.make_mlp(1)
    r = np.random.default_rng(4).normal(size=(3, 128, 128))
    a, _ = gpu_grads(M, scene, cams[0], mlp, r, (0, 0, 0))
    b, _ = gpu_grads(M, scene, cams[0], mlp, r, (0, 0, 0))
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def _backward_raw(M, R, scene_d, cam_s, capacity, gimg, mlp_params=None):
    """mgs_render_backward through the C ABI on a forward's buffers, with the given capacity."""
    L = M._lib
    n = scene_d.n
    g = {k: torch.full_like(scene_d.t[k], float("nan")) for k in KEYS}
    gs = L.mgs_gaussians_grad()
    gs.mean, gs.log_scale, gs.quat = (L.ptr(g[k]).value for k in ("mean", "log_scale", "quat"))
    gs.opacity_logit, gs.sh = L.ptr(g["opacity_logit"]).value, L.ptr(g["sh"]).value
    nb = L.C.c_size_t()
    L.check(L.lib().mgs_render_backward_workspace(n, R.tiles_x, R.tiles_y, capacity, int(mlp_params is not None),
                                                  L.C.byref(nb)))
    ws = torch.empty((nb.value + 255) // 256 * 64, dtype=torch.float32, device="cuda")
    dmlp = torch.full((L.MGS_MLP_PARAMS,), float("nan"), device="cuda") if mlp_params is not None else None
    use = mlp_params is not None
    L.check(L.lib().mgs_render_backward(
        L.C.byref(scene_d.struct), L.C.byref(cam_s), L.ptr(mlp_params) if use else None,
        L.ptr(R.phi) if use else None, L.ptr(R.omod) if use else None, L.C.byref(R.proj),
        L.ptr(R.tile_offsets), L.ptr(R.gids), capacity, L.ptr(R.aux), L.ptr(gimg), L.bg_array((0.1, 0.2, 0.3)),
        1 / 255, 0.99, L.ptr(ws), ws.numel() * 4, L.C.byref(gs), L.ptr(dmlp) if use else None, L.stream_ptr()))
    torch.cuda.synchronize()
    out = {k: g[k].cpu() for k in KEYS}
    if use:
        out["mlp"] = dmlp.cpu()
    return out


@pytest.mark.parametrize("with_mlp", [False, True])
def test_backward_after_overflowed_lists_is_zero(M, with_mlp):
    """A capacity below the forward's pair count means the lists overflowed: the backward reads
    no list (the work plan is empty) and every gradient is zero.  The same buffers with the full
    capacity give nonzero gradients, so the zeros come from the overflow rule."""
    say(f"test_backward_after_overflowed_lists_is_zero[{with_mlp}]")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    cam = cams[0]
    mlp = mgs_data.make_mlp(3) if with_mlp else None
    ds = M.DeviceScene(scene)
    dm = M.DeviceMLP(mlp) if with_mlp else None
    R = M.Renderer(ds.n, cam.width, cam.height)
    R.render(ds, cam, dm, bg=(0.1, 0.2, 0.3), want_aux=True, fused=False)
    P = R.pairs()
    assert 1000 < P <= R.capacity
    gimg = torch.as_tensor(np.random.default_rng(9).normal(size=(3, cam.height, cam.width)), dtype=torch.float32,
                           device="cuda")
    cam_s = M._lib.make_camera(cam)
    mp = dm.params if with_mlp else None
    full = _backward_raw(M, R, ds, cam_s, R.capacity, gimg, mp)
    over = _backward_raw(M, R, ds, cam_s, P - 1, gimg, mp)
    for k in full:
        assert torch.isfinite(full[k]).all() and torch.isfinite(over[k]).all(), k
        assert float(full[k].abs().max()) > 0, k
        assert float(over[k].abs().max()) == 0.0, k


def test_backward_with_no_pairs_is_zero(M):
    """A camera that sees no Gaussian: no pair, no work item, zero gradients."""
    say("test_backward_with_no_pairs_is_zero")
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    cam = mgs_data.look_at((0.0, 0.0, -3.0), target=(0.0, 0.0, -10.0), width=96, height=80, f=96.0)
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, cam.width, cam.height)
    R.render(ds, cam, bg=(0.1, 0.2, 0.3), want_aux=True)
    assert R.pairs() == 0
    gimg = torch.ones(3, cam.height, cam.width, device="cuda")
    out = _backward_raw(M, R, ds, M._lib.make_camera(cam), R.capacity, gimg)
    for k in out:
        assert float(out[k].abs().max()) == 0.0, k
