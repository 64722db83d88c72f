"""ctypes binding of libmgs.so (the C ABI declared in include/mgs.h).

Argument marshalling only: torch tensors supply device pointers and the
current HIP stream; every step of the render pass runs in the library's
kernels.  Importing this module fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# MGS_LIBRARY=checked loads libmgs_checked.so (the bounds-checked build of the same sources)
LIB_PATH = os.path.join(_PKG, "libmgs_checked.so" if os.environ.get("MGS_LIBRARY") == "checked" else "libmgs.so")

MGS_OK = 0
MGS_ERR_INVALID_ARG = -1
MGS_ERR_CAPACITY = -2
MGS_ERR_HIP = -3
MGS_ERR_UNSUPPORTED = -4
MGS_TILE = 16
MGS_MLP_PACKED_BYTES = 15360
MGS_SPLAT_FLOATS = 12
MGS_MLP_PARAMS = 5762
MLP_LAYOUT = (("W1", 0, (64, 22)), ("b1", 1408, (64,)), ("W2", 1472, (64, 64)), ("b2", 5568, (64,)),
              ("w_phi", 5632, (64,)), ("b_phi", 5696, ()), ("w_o", 5697, (64,)), ("b_o", 5761, ()))

EXPORTED = [
    "mgs_last_error", "mgs_version", "mgs_mlp_pack", "mgs_enhance", "mgs_project", "mgs_enhance_project",
    "mgs_bin_workspace", "mgs_bin", "mgs_blend_oit", "mgs_blend_oit_split_workspace", "mgs_blend_oit_split",
    "mgs_bin_sorted_workspace",
    "mgs_bin_sorted", "mgs_blend_sorted", "mgs_tile_sort_workspace", "mgs_tile_sort", "mgs_render_backward_workspace",
    "mgs_render_backward", "mgs_batch_workspace", "mgs_render_batch", "mgs_nvq_decode", "mgs_enhance_project_nvq",
    "mgs_project_weighted", "mgs_enhance_project_weighted", "mgs_mlp_f_pack", "mgs_enhance_project_mlp_f",
    "mgs_enhance_project_sh", "mgs_project_sortfree", "mgs_enhance_project_sortfree", "mgs_blend_sortfree",
    "mgs_blend_sortfree_split", "mgs_blend_oit_split_noalloc", "mgs_blend_census", "mgs_bounds_checked",
    "mgs_bounds_status", "mgs_check_capacity", "mgs_prune_workspace", "mgs_prune_vote", "mgs_prune_compact",
    "mgs_gather_planes",
]
MGS_NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024
# the appendix's MLP_f (hidden layers 256, 128, 64): name, offset, shape in the mgs.h layout
MLPF_LAYOUT = (("W1", 0, (256, 22)), ("b1", 5632, (256,)), ("W2", 5888, (128, 256)), ("b2", 38656, (128,)),
               ("W3", 38784, (64, 128)), ("b3", 46976, (64,)), ("w_phi", 47040, (64,)), ("b_phi", 47104, ()),
               ("w_o", 47105, (64,)), ("b_o", 47169, ()))
MGS_MLPF_PARAMS, MGS_MLPF_PACKED_BYTES = 47170, 104208
MGS_WEIGHT_EQ3, MGS_WEIGHT_NO_DEPTH, MGS_WEIGHT_NO_SCALE, MGS_WEIGHT_SORTFREE = 0, 1, 2, 3
MGS_NVQ_GROUPS, MGS_NVQ_DIM, MGS_NVQ_CODEWORDS = 5, 4, 1024
MGS_PRUNE_OPACITY, MGS_PRUNE_SCALE, MGS_PRUNE_BOTH = 1, 2, 3


class MgsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mgs error {code}: {msg}")
        self.code = code


class mgs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("near_z", C.c_float)]


class mgs_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("log_scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("sh", C.c_void_p)]


class mgs_gaussians_grad(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("log_scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("sh", C.c_void_p)]


class mgs_gaussians_nvq(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("codes", C.c_void_p), ("codebooks", C.c_void_p)]


class mgs_projected(C.Structure):
    _fields_ = [("splat", C.c_void_p), ("rect", C.c_void_p), ("n_tiles", C.c_void_p)]


class mgs_request(C.Structure):
    _fields_ = [("g", mgs_gaussians), ("packed_mlp", C.c_void_p), ("cam", mgs_camera), ("bg", C.c_float * 3),
                ("image", C.c_void_p)]


def load(path=None):
    """Open the library at ``path`` (default: the module's LIB_PATH as it is at call time)."""
    path = LIB_PATH if path is None else path
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2603_11531_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, u64, f32 = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_float
    P = C.POINTER
    sig = {
        "mgs_last_error": (C.c_char_p, []),
        "mgs_version": (C.c_char_p, []),
        "mgs_check_capacity": (i32, [vp, u64, P(C.c_uint64), vp]),
        "mgs_prune_workspace": (i32, [i64, P(C.c_size_t)]),
        "mgs_prune_vote": (i32, [vp, vp, i64, C.c_double, i32, vp, C.c_size_t, vp, vp, vp]),
        "mgs_prune_compact": (i32, [vp, i64, C.c_uint32, vp, C.c_size_t, vp, vp, vp]),
        "mgs_gather_planes": (i32, [vp, i64, i32, vp, vp, i64, vp, i64, vp]),
        "mgs_mlp_pack": (i32, [vp, vp, vp]),
        "mgs_enhance": (i32, [P(mgs_gaussians), P(mgs_camera), vp, vp, vp, vp]),
        "mgs_project": (i32, [P(mgs_gaussians), P(mgs_camera), vp, vp, i32, f32, P(mgs_projected), vp]),
        "mgs_enhance_project": (i32, [P(mgs_gaussians), P(mgs_camera), vp, i32, f32, P(mgs_projected), vp, vp, vp]),
        "mgs_mlp_f_pack": (i32, [vp, vp, vp]),
        "mgs_enhance_project_sh": (i32, [P(mgs_gaussians), i32, P(mgs_camera), vp, i32, f32, P(mgs_projected), vp,
                                         vp, vp]),
        "mgs_enhance_project_mlp_f": (i32, [P(mgs_gaussians), P(mgs_camera), vp, i32, f32, P(mgs_projected), vp, vp,
                                            vp]),
        "mgs_project_weighted": (i32, [P(mgs_gaussians), P(mgs_camera), vp, vp, i32, f32, i32, P(mgs_projected),
                                       vp]),
        "mgs_enhance_project_weighted": (i32, [P(mgs_gaussians), P(mgs_camera), vp, i32, f32, i32,
                                               P(mgs_projected), vp, vp, vp]),
        "mgs_project_sortfree": (i32, [P(mgs_gaussians), P(mgs_camera), vp, vp, vp, i32, f32, P(mgs_projected),
                                       vp]),
        "mgs_enhance_project_sortfree": (i32, [P(mgs_gaussians), P(mgs_camera), vp, vp, vp, i32, f32,
                                               P(mgs_projected), vp, vp, vp]),
        "mgs_blend_sortfree": (i32, [P(mgs_projected), vp, vp, P(mgs_camera), i32, P(C.c_float), f32, f32, f32, vp,
                                     vp, vp]),
        "mgs_blend_sortfree_split": (i32, [P(mgs_projected), vp, vp, vp, u64, P(mgs_camera), i32, P(C.c_float), f32,
                                           f32, f32, vp, C.c_size_t, vp, vp, vp]),
        "mgs_blend_oit_split_noalloc": (i32, [P(mgs_projected), vp, vp, vp, u64, P(mgs_camera), i32, P(C.c_float),
                                              f32, f32, vp, vp, vp]),
        "mgs_blend_census": (i32, [P(mgs_projected), vp, vp, vp, u64, P(mgs_camera), f32, vp, vp]),
        "mgs_bounds_checked": (i32, []),
        "mgs_bounds_status": (i32, [P(C.c_uint32), i32]),
        "mgs_bin_workspace": (i32, [i64, i32, i32, u64, P(C.c_size_t)]),
        "mgs_bin": (i32, [P(mgs_projected), i64, i32, i32, vp, C.c_size_t, vp, vp, u64, vp, vp]),
        "mgs_blend_oit": (i32, [P(mgs_projected), vp, vp, P(mgs_camera), i32, P(C.c_float), f32, f32, vp, vp,
                                vp]),
        "mgs_blend_oit_split_workspace": (i32, [i32, i32, u64, P(C.c_size_t)]),
        "mgs_blend_oit_split": (i32, [P(mgs_projected), vp, vp, vp, u64, P(mgs_camera), i32, P(C.c_float), f32, f32,
                                      vp, C.c_size_t, vp, vp, vp]),
        "mgs_bin_sorted_workspace": (i32, [i64, i32, i32, u64, P(C.c_size_t)]),
        "mgs_bin_sorted": (i32, [P(mgs_projected), i64, i32, i32, vp, C.c_size_t, vp, vp, u64, vp, vp]),
        "mgs_tile_sort_workspace": (i32, [i32, i32, u64, P(C.c_size_t)]),
        "mgs_tile_sort": (i32, [P(mgs_projected), i64, vp, vp, i32, i32, u64, vp, vp, C.c_size_t, vp]),
        "mgs_blend_sorted": (i32, [P(mgs_projected), vp, vp, P(mgs_camera), i32, P(C.c_float), f32, f32, f32,
                                   vp, vp]),
        "mgs_nvq_decode": (i32, [P(mgs_gaussians_nvq), vp, vp, vp, vp, vp]),
        "mgs_enhance_project_nvq": (i32, [P(mgs_gaussians_nvq), P(mgs_camera), vp, i32, f32, P(mgs_projected), vp,
                                          vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    lib.mgs_batch_workspace.restype = i32
    lib.mgs_batch_workspace.argtypes = [i64, i64, u64, P(C.c_size_t)]
    lib.mgs_render_batch.restype = i32
    lib.mgs_render_batch.argtypes = [vp, vp, i64, i64, u64, f32, f32, vp, C.c_size_t, vp, vp, vp]
    lib.mgs_render_backward_workspace.restype = i32
    lib.mgs_render_backward_workspace.argtypes = [i64, i32, i32, u64, i32, P(C.c_size_t)]
    lib.mgs_render_backward.restype = i32
    lib.mgs_render_backward.argtypes = [
        P(mgs_gaussians), P(mgs_camera), vp, vp, vp, P(mgs_projected), vp, vp, u64, vp, vp, P(C.c_float), f32,
        f32, vp, C.c_size_t, P(mgs_gaussians_grad), vp, vp]
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def check(code):
    if code != MGS_OK:
        raise MgsError(code, lib().mgs_last_error().decode())
    return code


def ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def make_camera(cam) -> mgs_camera:
    c = mgs_camera()
    for i, v in enumerate(list(map(float, cam.R.reshape(-1)))):
        c.R[i] = v
    for i, v in enumerate(list(map(float, cam.t.reshape(-1)))):
        c.t[i] = v
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height, c.near_z = int(cam.width), int(cam.height), float(cam.near)
    return c


def make_gaussians(scene) -> mgs_gaussians:
    """``scene`` = dict of device float32 tensors in the SoA layout of mgs.h."""
    g = mgs_gaussians()
    g.n = int(scene["opacity_logit"].numel())
    g.mean, g.log_scale, g.quat = (ptr(scene[k]).value for k in ("mean", "log_scale", "quat"))
    g.opacity_logit, g.sh = ptr(scene["opacity_logit"]).value, ptr(scene["sh"]).value
    return g


def make_gaussians_nvq(q) -> mgs_gaussians_nvq:
    """``q`` = dict of device tensors: mean [3][N] float32, codes [5][N] int16 (uint16 bits),
    codebooks [5][1024][4] float32."""
    g = mgs_gaussians_nvq()
    g.n = int(q["codes"].shape[1])
    g.mean, g.codes, g.codebooks = (ptr(q[k]).value for k in ("mean", "codes", "codebooks"))
    return g


def make_projected(splat, rect, n_tiles) -> mgs_projected:
    p = mgs_projected()
    p.splat, p.rect, p.n_tiles = ptr(splat).value, ptr(rect).value, ptr(n_tiles).value
    return p


def bg_array(bg):
    return (C.c_float * 3)(*[float(v) for v in bg])
