"""The appendix's enhancement network MLP_f (ReLU layers 256, 128, 64) fused with the
projection, through the C ABI, against the FP64 oracle (its BF16 emulation and the plain
FP64 network).  Tolerances as for the two-layer MLP: per-Gaussian phi / m within 2e-2
(relative to max phi) / 1e-2 of the emulation with a median below 1e-5 (rare bf16 rounding
flips aside), and the image within 1e-4 of the emulation's admissible results on all but
1/2000 of the pixels, PSNR >= 50 dB against the FP64 oracle."""
import numpy as np
import pytest
import torch

import mgs_data
import oracle as O
from gpu_helpers import compare_oit_image, psnr, say

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11531_amd as M
    M._lib.lib()
    return M


def _oracle(scene, cam, mlp, bf16):
    camt = O.camera_tensors(cam)
    p = O.scene_params(scene)
    act = O.activate(p)
    _, _, P = O.camera_space(p["mean"], camt)
    with torch.no_grad():
        phi, m = O.enhance(O.mlp_features(P, act["s"], act["q"], p["sh"]), O.mlp_params(mlp), bf16=bf16)
        return phi, m, O.project(p, camt, phi, m), camt


@pytest.mark.parametrize("n", [20000, 1037, 50])
def test_mlp_f_enhance_project_matches_oracle(M, n):
    say(f"test_mlp_f_enhance_project_matches_oracle[{n}]")
    scene = mgs_data.make_scene_unbounded(n, 5)
    cam = mgs_data.circle_poses(8, 10.0, 200, 132, f=200.0)[3]
    mlp = mgs_data.make_mlp_f(6)
    ds, dm = M.DeviceScene(scene), M.DeviceMLPF(mlp)
    R = M.Renderer(ds.n, cam.width, cam.height)
    img = R.render(ds, cam, dm).double().cpu()
    torch.cuda.synchronize()
    phi_g, m_g = R.phi.double().cpu(), R.omod.double().cpu()
    phi_e, m_e, pr_e, camt = _oracle(scene, cam, mlp, bf16=True)
    phi_f, m_f, pr_f, _ = _oracle(scene, cam, mlp, bf16=False)
    e_phi, e_m = float((phi_g - phi_e).abs().max()), float((m_g - m_e).abs().max())
    say(f"  phi / m vs emulation {e_phi:.2e} / {e_m:.2e}; vs fp64 {float((phi_g - phi_f).abs().max()):.2e} / "
        f"{float((m_g - m_f).abs().max()):.2e}")
    assert e_phi < 2e-2 * float(phi_e.abs().max()) and e_m < 1e-2
    assert float((phi_g - phi_e).abs().median()) < 1e-5 and float((m_g - m_e).abs().median()) < 1e-5
    _, _, V, flagged = O.render_oit(pr_e, camt, np.array((0.0, 0.0, 0.0)), mode="binned", variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    ref_f, _ = O.render_oit(pr_f, camt, np.array((0.0, 0.0, 0.0)), mode="binned")
    e64, ps = float((img - ref_f).abs().max()), psnr(img, ref_f)
    say(f"  image vs emulation max {err:.3e} fails {nfail}; vs fp64 max {e64:.3e} psnr {ps:.1f} dB")
    assert nfail <= max(2, img[0].numel() // 2000)
    assert e64 <= 2e-2 and ps >= 50.0


def test_mlp_f_is_deterministic_and_differs_from_the_two_layer_network(M):
    say("test_mlp_f_is_deterministic_and_differs_from_the_two_layer_network")
    scene = mgs_data.make_scene_unbounded(30001, 8)
    cam = mgs_data.circle_poses(8, 10.0, 240, 160, f=240.0)[5]
    ds = M.DeviceScene(scene)
    dmf = M.DeviceMLPF(mgs_data.make_mlp_f(9))
    a = M.Renderer(ds.n, cam.width, cam.height)
    b = M.Renderer(ds.n, cam.width, cam.height)
    ia = a.render(ds, cam, dmf).clone()
    ib = b.render(ds, cam, dmf).clone()
    torch.cuda.synchronize()
    assert torch.equal(ia, ib) and torch.equal(a.phi, b.phi) and torch.equal(a.splat, b.splat)
    c = M.Renderer(ds.n, cam.width, cam.height)
    ic = c.render(ds, cam, M.DeviceMLP(mgs_data.make_mlp(9)), fused=True)
    torch.cuda.synchronize()
    assert not torch.equal(ia, ic)


def test_mlp_f_rejects_bad_arguments(M):
    from paper_2603_11531_amd import _lib as L
    say("test_mlp_f_rejects_bad_arguments")
    scene = mgs_data.make_scene_unbounded(100, 2)
    ds = M.DeviceScene(scene)
    R = M.Renderer(ds.n, 64, 64)
    cam_s = L.make_camera(mgs_data.look_at((0.0, 0.0, -4.0), width=64, height=64))
    lib = L.lib()
    dm = M.DeviceMLPF(mgs_data.make_mlp_f(1))
    rc = lib.mgs_enhance_project_mlp_f(L.C.byref(ds.struct), L.C.byref(cam_s), None, L.MGS_TILE, 1 / 255,
                                       L.C.byref(R.proj), L.ptr(R.phi), L.ptr(R.omod), None)
    assert rc == L.MGS_ERR_INVALID_ARG
    rc = lib.mgs_enhance_project_mlp_f(L.C.byref(ds.struct), L.C.byref(cam_s), L.ptr(dm.packed), 8, 1 / 255,
                                       L.C.byref(R.proj), L.ptr(R.phi), L.ptr(R.omod), None)
    assert rc == L.MGS_ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        M.DeviceMLPF(mgs_data.make_mlp(1))          # a two-layer network does not fit the layout
