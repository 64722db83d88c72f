"""Worker of tests/test_gpu_bounds.py: drives the render paths through the library named by
MGS_LIBRARY (the bounds-checked build when "checked"), prints the bounds flags and saves the
images to the .npz given on the command line."""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import mgs_data  # noqa: E402
import paper_2603_11531_amd as M  # noqa: E402
from paper_2603_11531_amd import serve  # noqa: E402
from paper_2603_11531_amd.autograd import render as diff_render  # noqa: E402


def cases():
    """(name, scene, camera, mlp or None, extra render arguments)."""
    out = []
    scene, cams, _, _ = mgs_data.make_config("small", seed=0)
    out.append(("small", scene, cams[0], None, {}))
    out.append(("small_sorted", scene, cams[0], None, {"sorted_path": True}))
    sc = mgs_data.make_scene_uniform(800, 7, ls_mu=-2.8)
    for W, H in ((33, 17), (1, 1), (250, 130)):
        out.append((f"ragged_{W}x{H}", sc, mgs_data.look_at((0.2, -0.4, -3.2), width=W, height=H, f=float(max(W, 8))),
                    None, {}))
    empty = {k: v[..., :0].copy() for k, v in mgs_data.make_scene_uniform(1, 0).items()}
    out.append(("empty", empty, mgs_data.look_at((0, 0, -4), width=40, height=24, f=40.0), None, {}))
    # one tile whose list is longer than 255 ranges of 2,048 (the split plan's long-list rule), and
    # the per-tile depth sort of that list (its workspace path)
    dense = mgs_data.make_scene_uniform(540_000, 21, half=0.5, ls_mu=-4.5)
    cam16 = mgs_data.look_at((0.0, 0.0, -4.0), width=16, height=16, f=16.0)
    out.append(("one_tile_540k", dense, cam16, None, {}))
    out.append(("one_tile_540k_tile_sort", dense, cam16, None, {"sorted_path": "tile_sort"}))
    # a view of two split-plan chunks (14,400 tiles), dense middle tiles split
    big = mgs_data.make_scene_uniform(100_000, 31, ls_mu=-3.1)
    out.append(("view_2560x1440", big, mgs_data.look_at((0.1, 0.2, -4.0), width=2560, height=1440, f=1536.0), None,
                {}))
    ub = mgs_data.make_scene_unbounded(30000, 8)
    cam = mgs_data.circle_poses(8, 10.0, 240, 160, f=240.0)[5]
    mlp = mgs_data.make_mlp(9)
    out.append(("mlp_fused", ub, cam, mlp, {"fused": True}))
    out.append(("mlp_sorted", ub, cam, mlp, {"fused": True, "sorted_path": True}))
    out.append(("mlp_tile_sort", ub, cam, mlp, {"fused": True, "sorted_path": "tile_sort"}))
    sig, bet = mgs_data.make_sortfree_params(30000, 3)
    out.append(("eq1", ub, cam, mlp, {"fused": True, "w_bg": 0.4,
                                      "sortfree": (torch.as_tensor(sig).cuda(), torch.as_tensor(bet).cuda())}))
    return out


def main(path):
    L = M._lib
    lib = L.lib()
    images = {}
    for name, scene, cam, mlp, kw in cases():
        ds = M.DeviceScene(scene)
        R = M.Renderer(ds.n, cam.width, cam.height)
        dm = M.DeviceMLP(mlp) if mlp is not None else None
        images[name] = R.render(ds, cam, dm, bg=(0.1, 0.2, 0.3), **kw).cpu().numpy().copy()
    # batched serving: three scenes, four resolutions in one launch
    reg = serve.SceneRegistry()
    reg.add("a", mgs_data.make_scene_uniform(3000, 31), mgs_data.make_mlp(40))
    reg.add("b", mgs_data.make_scene_uniform(7777, 32), None)
    slot = serve.BatchSlot(max_gaussians=200_000, max_tiles=4 * 8160, capacity=4_000_000, use_graphs=False)
    reqs = []
    for k, (name, (W, H)) in enumerate(zip(["a", "b", "a", "b"], [(96, 64), (130, 77), (200, 120), (33, 17)])):
        c = mgs_data.look_at((0.7 * np.sin(k), -0.3 * np.cos(k), -3.5 - 0.2 * k), width=W, height=H, f=float(W))
        r = serve.Request(rid=k, scene=name, cam=c, arrival=0.0, bg=(0.1 * k, 0.2, 0.05 * k))
        r.image = torch.zeros(3, H, W, device="cuda")
        reqs.append(r)
    slot.launch(reqs, reg)
    slot.done_event.synchronize()
    for r in reqs:
        images[f"batch_{r.rid}"] = r.image.cpu().numpy().copy()
    # pruning: two iterations' votes (the same candidates twice: more than I_prune v = 1), the
    # compaction and the gather of every attribute plane
    from paper_2603_11531_amd import prune
    sc = mgs_data.make_scene_uniform(20_000, 41)
    ts = {k: torch.from_numpy(np.ascontiguousarray(sc[k], np.float32)).cuda()
          for k in ("mean", "log_scale", "quat", "opacity_logit", "sh")}
    pr = prune.Pruner(20_000, interval=2, v=0.5)
    for _ in range(2):
        pr.vote(ts["opacity_logit"], ts["log_scale"])
    pruned, kept = pr.prune(ts)
    images["prune_kept"] = kept.cpu().numpy().copy()
    for k, v in pruned.items():
        images[f"prune_{k}"] = v.cpu().numpy().copy()
    # backward on dense tile lists, with the MLP
    scene = mgs_data.make_scene_uniform(40000, 31, half=2.2, ls_mu=-2.5)
    cam = mgs_data.look_at((0.1, -0.1, -4.0), width=96, height=96, f=96.0)
    keys = ("mean", "log_scale", "quat", "opacity_logit", "sh")
    params = {k: torch.tensor(np.ascontiguousarray(scene[k]), device="cuda", requires_grad=True) for k in keys}
    dmlp = M.DeviceMLP(mgs_data.make_mlp(32))
    mp = dmlp.params.clone().requires_grad_(True)
    img = diff_render(params, cam, mp, (0.1, 0.3, 0.2))
    (img * torch.linspace(-1, 1, img.numel(), device="cuda").reshape(img.shape)).sum().backward()
    images["backward_mean_grad"] = params["mean"].grad.cpu().numpy().copy()
    images["backward_mlp_grad"] = mp.grad.cpu().numpy().copy()
    torch.cuda.synchronize()
    flags = L.C.c_uint32()
    L.check(lib.mgs_bounds_status(L.C.byref(flags), 1))
    np.savez(path, **images)
    print(f"checked={lib.mgs_bounds_checked()} flags=0x{flags.value:x} cases={len(images)}", flush=True)
    if lib.mgs_bounds_checked():
        # a planted inconsistency: the pair count 8 below the lists' extent.  Every list read
        # stays inside the gids buffer (its capacity holds the true lists), so no access can
        # leave an allocation; the checked blend must report the reads past the count.
        scene, cams, _, _ = mgs_data.make_config("small", seed=0)
        ds = M.DeviceScene(scene)
        R = M.Renderer(ds.n, cams[0].width, cams[0].height)
        R.render(ds, cams[0])
        P = R.pairs()
        assert P > 16 and R.capacity >= P
        R.n_pairs.fill_(P - 8)
        R.blend_oit(L.make_camera(cams[0]))
        torch.cuda.synchronize()
        L.check(lib.mgs_bounds_status(L.C.byref(flags), 1))
        print(f"planted=0x{flags.value:x}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
