"""Vector-quantised attributes (Sec. 3.2): the codebook decode and the fused enhance +
project that reads through the codebooks, against the oracle's decode (bit-exact), the
float32 path on the decoded attributes (bit-exact) and the FP64 oracle image."""
import numpy as np
import pytest
import torch

import mgs_data
import oracle as O
from gpu_helpers import compare_oit_image, oracle_project, psnr, say

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11531_amd as M
    M._lib.lib()
    return M


def _nvq(n, seed):
    return mgs_data.make_nvq(mgs_data.make_scene_unbounded(n, seed), seed + 100)


def test_decode_is_the_oracle_lookup(M):
    say("test_decode_is_the_oracle_lookup")
    for n in (1, 63, 4099):
        q = _nvq(n, 1)
        if n == 4099:
            q["codes"][:, ::7] |= np.uint16(0x8000)          # out-of-range codes are taken modulo 1024
        ds = M.DeviceNVQ(q).decode()
        torch.cuda.synchronize()
        ref = O.nvq.decode(q["codes"] % 1024, q["codebooks"], q["mean"])
        for k in ("mean", "log_scale", "quat", "opacity_logit", "sh"):
            assert np.array_equal(ds.t[k].cpu().numpy(), ref[k]), (n, k)


def test_fused_nvq_equals_float32_path_on_decoded_attributes(M):
    say("test_fused_nvq_equals_float32_path_on_decoded_attributes")
    q = _nvq(50_000, 2)
    cam = mgs_data.circle_poses(8, 10.0, 320, 200, f=320.0)[1]
    mlp = mgs_data.make_mlp(3)
    dm = M.DeviceMLP(mlp)
    dq = M.DeviceNVQ(q)
    ds = M.DeviceScene(O.nvq.decode(q["codes"], q["codebooks"], q["mean"]))
    cs = M._lib.make_camera(cam)
    out = []
    for scene, fn in ((dq, "enhance_project_nvq"), (ds, "enhance_project")):
        R = M.Renderer(scene.n, cam.width, cam.height)
        getattr(R, fn)(scene, cs, dm)
        torch.cuda.synchronize()
        out.append({k: getattr(R, k).clone() for k in ("splat", "rect", "n_tiles", "phi", "omod")})
    for k in out[0]:
        assert torch.equal(out[0][k], out[1][k]), k


def test_nvq_render_matches_oracle(M):
    say("test_nvq_render_matches_oracle")
    q = _nvq(20_000, 4)
    cam = mgs_data.circle_poses(8, 10.0, 200, 132, f=200.0)[5]
    mlp = mgs_data.make_mlp(6)
    bg = (0.1, 0.0, 0.2)
    R = M.Renderer(q["codes"].shape[1], cam.width, cam.height)
    img = R.render(M.DeviceNVQ(q), cam, M.DeviceMLP(mlp), bg=bg).double().cpu()
    scene = O.nvq.decode(q["codes"], q["codebooks"], q["mean"])
    pr_e, camt = oracle_project(scene, cam, mlp=mlp, bf16=True)
    _, _, V, flagged = O.render_oit(pr_e, camt, np.array(bg), mode="binned", variants=True)
    err, nfail = compare_oit_image(img, V, flagged, TOL)
    pr_f, _ = oracle_project(scene, cam, mlp=mlp, bf16=False)
    ref_f, _ = O.render_oit(pr_f, camt, np.array(bg), mode="binned")
    e64, ps = float((img - ref_f).abs().max()), psnr(img, ref_f)
    say(f"  vs bf16-emulation: max {err:.3e} fails {nfail}; vs fp64: max {e64:.3e} psnr {ps:.1f} dB")
    assert e64 <= 2e-2 and ps >= 50.0
    assert nfail <= max(2, img[0].numel() // 2000)
