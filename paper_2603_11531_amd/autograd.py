"""torch.autograd.Function over the C ABI: forward = enhance -> project -> bin -> OIT
blend (with aux), backward = mgs_render_backward.

Gradients flow to the raw Gaussian attributes (mean, log_scale, quat,
opacity_logit, sh; SoA float32 device tensors as in include/mgs.h) and, when
the MLP is on, to its flat parameter tensor (MGS_MLP_PARAMS floats).
"""
from __future__ import annotations

import torch

from . import _lib as L
from .render import ALPHA_MAX, ALPHA_MIN, DeviceScene, Renderer


class _State:
    """Forward buffers kept for one backward call."""


class MGSRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cam, bg, mean, log_scale, quat, opacity_logit, sh, mlp_params):
        dev = mean.device
        scene = DeviceScene.from_tensors(dict(mean=mean.detach(), log_scale=log_scale.detach(), quat=quat.detach(),
                                              opacity_logit=opacity_logit.detach(), sh=sh.detach()))
        if scene.sh_degree != 1:
            raise ValueError("the backward pass differentiates first-order SH only")
        R = Renderer(scene.n, cam.width, cam.height, device=dev)
        cam_s = L.make_camera(cam)
        use_mlp = mlp_params is not None
        packed = None
        if use_mlp:
            params = mlp_params.detach().contiguous()
            packed = torch.empty(L.MGS_MLP_PACKED_BYTES // 4, dtype=torch.float32, device=dev)
            L.check(L.lib().mgs_mlp_pack(L.ptr(params), L.ptr(packed), L.stream_ptr()))
            L.check(L.lib().mgs_enhance(L.C.byref(scene.struct), L.C.byref(cam_s), L.ptr(packed), L.ptr(R.phi),
                                        L.ptr(R.omod), L.stream_ptr()))
        R.project(scene, cam_s, use_mlp=use_mlp)
        R.bin()
        P = R.pairs()
        if P > R.capacity:
            R.ensure_capacity(int(P * 1.25) + 1024)
            R.bin()
        R.blend_oit(cam_s, bg, want_aux=True)
        st = _State()
        st.R, st.scene, st.cam_s, st.bg, st.use_mlp = R, scene, cam_s, tuple(float(v) for v in bg), use_mlp
        st.mlp_params = mlp_params.detach().contiguous() if use_mlp else None
        ctx.st = st
        return R.image.clone()

    @staticmethod
    def backward(ctx, gimg):
        st = ctx.st
        R, scene = st.R, st.scene
        n = scene.n
        dev = R.device
        g = {k: torch.empty_like(scene.t[k]) for k in DeviceScene.KEYS}
        gs = L.mgs_gaussians_grad()
        gs.mean, gs.log_scale, gs.quat = (L.ptr(g[k]).value for k in ("mean", "log_scale", "quat"))
        gs.opacity_logit, gs.sh = L.ptr(g["opacity_logit"]).value, L.ptr(g["sh"]).value
        nb = L.C.c_size_t()
        L.check(L.lib().mgs_render_backward_workspace(n, R.tiles_x, R.tiles_y, R.capacity, int(st.use_mlp),
                                                      L.C.byref(nb)))
        ws = torch.empty((nb.value + 255) // 256 * 64, dtype=torch.float32, device=dev)
        dmlp = torch.zeros(L.MGS_MLP_PARAMS, dtype=torch.float32, device=dev) if st.use_mlp else None
        gimg = gimg.contiguous().to(torch.float32)
        L.check(L.lib().mgs_render_backward(
            L.C.byref(scene.struct), L.C.byref(st.cam_s), L.ptr(st.mlp_params),
            L.ptr(R.phi) if st.use_mlp else None, L.ptr(R.omod) if st.use_mlp else None,
            L.C.byref(R.proj), L.ptr(R.tile_offsets), L.ptr(R.gids), R.capacity, L.ptr(R.aux), L.ptr(gimg),
            L.bg_array(st.bg), ALPHA_MIN, ALPHA_MAX, L.ptr(ws), ws.numel() * 4, L.C.byref(gs), L.ptr(dmlp),
            L.stream_ptr()))
        return None, None, g["mean"], g["log_scale"], g["quat"], g["opacity_logit"], g["sh"], dmlp


def render(params, cam, mlp_params=None, bg=(0.0, 0.0, 0.0)):
    """Differentiable OIT render of one view.  ``params``: dict of SoA device tensors."""
    return MGSRender.apply(cam, tuple(bg), params["mean"], params["log_scale"], params["quat"],
                           params["opacity_logit"], params["sh"], mlp_params)
