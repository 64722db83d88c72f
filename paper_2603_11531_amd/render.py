"""Python front end of the render pass: device buffers + the C-ABI calls in order.

Everything numeric runs in libmgs.so; this module allocates torch device
tensors, passes their pointers and the current stream, and manages the pair
capacity of the tile lists (the only data-dependent size of the pass).
"""
from __future__ import annotations


import numpy as np
import torch

from . import _lib as L

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_STOP = 1e-4


def _u32_to_i64(t):
    return t.to(torch.int64) & 0xFFFFFFFF


class DeviceScene:
    """Gaussian attributes resident in device memory (SoA float32, see mgs.h)."""

    KEYS = ("mean", "log_scale", "quat", "opacity_logit", "sh")

    # SH planes (3 per coefficient) -> SH order
    SH_DEGREE = {3: 0, 12: 1, 27: 2, 48: 3}

    def __init__(self, scene, device="cuda"):
        self.t = {k: torch.as_tensor(np.ascontiguousarray(scene[k], dtype=np.float32)).to(device)
                  for k in self.KEYS}
        self.n = int(self.t["opacity_logit"].numel())
        self.sh_degree = self._degree(self.t["sh"])
        self.struct = L.make_gaussians(self.t)

    @classmethod
    def _degree(cls, sh):
        planes = int(sh.shape[0]) if sh.dim() == 2 else 12
        if planes not in cls.SH_DEGREE:
            raise ValueError(f"{planes} SH planes: expected 3 (d + 1)^2 for an order d in 0..3")
        return cls.SH_DEGREE[planes]

    @classmethod
    def from_tensors(cls, tensors):
        obj = cls.__new__(cls)
        obj.t = {k: tensors[k].contiguous() for k in cls.KEYS}
        obj.n = int(obj.t["opacity_logit"].numel())
        obj.sh_degree = cls._degree(obj.t["sh"])
        obj.struct = L.make_gaussians(obj.t)
        return obj

    def nbytes(self):
        return sum(v.numel() * 4 for v in self.t.values())


class DeviceNVQ:
    """A vector-quantised scene resident in device memory (mgs_gaussians_nvq): float32
    positions, five uint16 codes per Gaussian and the five 1024 x 4 codebooks."""

    def __init__(self, q, device="cuda"):
        codes = np.ascontiguousarray(q["codes"], dtype=np.uint16).view(np.int16)   # torch has no uint16 ops
        self.t = {"mean": torch.as_tensor(np.ascontiguousarray(q["mean"], dtype=np.float32)).to(device),
                  "codes": torch.as_tensor(codes).to(device),
                  "codebooks": torch.as_tensor(np.ascontiguousarray(q["codebooks"], dtype=np.float32)).to(device)}
        self.n = int(self.t["codes"].shape[1])
        self.struct = L.make_gaussians_nvq(self.t)

    def nbytes(self):
        return sum(v.numel() * v.element_size() for v in self.t.values())

    def decode(self, stream=None):
        """mgs_nvq_decode into a new DeviceScene (float32 SoA planes)."""
        dev = self.t["mean"].device
        planes = {"mean": self.t["mean"],
                  "log_scale": torch.empty(3, self.n, dtype=torch.float32, device=dev),
                  "quat": torch.empty(4, self.n, dtype=torch.float32, device=dev),
                  "opacity_logit": torch.empty(self.n, dtype=torch.float32, device=dev),
                  "sh": torch.empty(12, self.n, dtype=torch.float32, device=dev)}
        L.check(L.lib().mgs_nvq_decode(L.C.byref(self.struct), L.ptr(planes["log_scale"]), L.ptr(planes["quat"]),
                                       L.ptr(planes["opacity_logit"]), L.ptr(planes["sh"]), L.stream_ptr(stream)))
        return DeviceScene.from_tensors(planes)


class DeviceMLP:
    """MLP parameters on the device (one float32 array, layout of mgs.h) plus the
    packed bf16 MFMA operands that mgs_enhance reads."""

    def __init__(self, mlp, device="cuda"):
        flat = np.zeros(L.MGS_MLP_PARAMS, np.float32)
        for name, off, shape in L.MLP_LAYOUT:
            v = np.asarray(mlp[name], np.float32).reshape(-1)
            flat[off:off + v.size] = v
        self.params = torch.as_tensor(flat).to(device)
        self.packed = torch.empty(L.MGS_MLP_PACKED_BYTES // 4, dtype=torch.float32, device=device)
        self.repack()

    def repack(self, stream=None):
        L.check(L.lib().mgs_mlp_pack(L.ptr(self.params), L.ptr(self.packed), L.stream_ptr(stream)))

    @staticmethod
    def unflatten(flat):
        """Split a float array in the mgs.h MLP layout into named numpy arrays."""
        flat = np.asarray(flat)
        return {name: flat[off:off + int(np.prod(shape)) if shape else off + 1].reshape(shape)
                for name, off, shape in L.MLP_LAYOUT}


class DeviceMLPF:
    """The appendix's MLP_f (hidden layers 256, 128, 64) on the device: parameters in the
    mgs.h layout plus the packed bf16 operands that mgs_enhance_project_mlp_f reads."""

    def __init__(self, mlp, device="cuda"):
        flat = np.zeros(L.MGS_MLPF_PARAMS, np.float32)
        for name, off, shape in L.MLPF_LAYOUT:
            v = np.asarray(mlp[name], np.float32).reshape(-1)
            if v.size != max(1, int(np.prod(shape))):
                raise ValueError(f"MLP_f parameter {name}: {v.size} values, layout wants shape {shape}")
            flat[off:off + v.size] = v
        self.params = torch.as_tensor(flat).to(device)
        self.packed = torch.empty(L.MGS_MLPF_PACKED_BYTES // 4, dtype=torch.float32, device=device)
        L.check(L.lib().mgs_mlp_f_pack(L.ptr(self.params), L.ptr(self.packed), None))


class Renderer:
    """Reusable buffers for one (N, W, H) shape; one call per stage or ``render``."""

    def __init__(self, n, width, height, device="cuda", capacity=None):
        self.device = torch.device(device)
        self.n, self.W, self.H = int(n), int(width), int(height)
        self.tiles_x = (self.W + L.MGS_TILE - 1) // L.MGS_TILE
        self.tiles_y = (self.H + L.MGS_TILE - 1) // L.MGS_TILE
        self.T = self.tiles_x * self.tiles_y
        nn = max(1, self.n)
        self.splat = torch.empty(nn, L.MGS_SPLAT_FLOATS, dtype=torch.float32, device=self.device)
        self.rect = torch.empty(nn, 2, dtype=torch.int32, device=self.device)
        self.n_tiles = torch.empty(nn, dtype=torch.int32, device=self.device)
        self.phi = torch.empty(nn, dtype=torch.float32, device=self.device)
        self.omod = torch.empty(nn, dtype=torch.float32, device=self.device)
        # zero-initialised so a blend after an overflowed bin reads empty lists, never garbage
        self.tile_offsets = torch.zeros(self.T + 1, dtype=torch.int32, device=self.device)
        self.n_pairs = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.image = torch.empty(3, self.H, self.W, dtype=torch.float32, device=self.device)
        self.aux = None
        self.proj = L.make_projected(self.splat, self.rect, self.n_tiles)
        self.capacity = 0
        self.gids = None
        self.ws = None
        self.ws_sorted = None
        self.ws_split = None
        self.ws_tsort, self.ws_tsort_cap = None, -1
        self.ensure_capacity(capacity if capacity is not None else max(1024, 4 * self.n))

    # -- capacity -----------------------------------------------------------
    def ensure_capacity(self, cap, sorted_path=False):
        cap = int(cap)
        lib = L.lib()
        if cap > self.capacity or self.gids is None:
            self.capacity = cap
            self.gids = torch.zeros(max(1, cap), dtype=torch.int32, device=self.device)
            self.ws = None
            self.ws_sorted = None
            self.ws_split = None
        if self.ws_split is None and not sorted_path:
            nb = L.C.c_size_t()
            L.check(lib.mgs_blend_oit_split_workspace(self.tiles_x, self.tiles_y, self.capacity, L.C.byref(nb)))
            self.ws_split = torch.empty((nb.value + 255) // 256 * 64, dtype=torch.float32, device=self.device)
        if self.ws is None and not sorted_path:
            nb = L.C.c_size_t()
            L.check(lib.mgs_bin_workspace(self.n, self.tiles_x, self.tiles_y, self.capacity, L.C.byref(nb)))
            self.ws = torch.empty((nb.value + 255) // 256 * 64, dtype=torch.float32, device=self.device)
        if self.ws_sorted is None and sorted_path:
            nb = L.C.c_size_t()
            L.check(lib.mgs_bin_sorted_workspace(self.n, self.tiles_x, self.tiles_y, self.capacity,
                                                 L.C.byref(nb)))
            self.ws_sorted = torch.empty((nb.value + 255) // 256 * 64, dtype=torch.float32, device=self.device)

    # -- stages -------------------------------------------------------------
    def enhance(self, scene: DeviceScene, cam_s, mlp: DeviceMLP, stream=None):
        L.check(L.lib().mgs_enhance(L.C.byref(scene.struct), L.C.byref(cam_s), L.ptr(mlp.packed),
                                    L.ptr(self.phi), L.ptr(self.omod), L.stream_ptr(stream)))

    def project(self, scene: DeviceScene, cam_s, use_mlp=False, alpha_min=ALPHA_MIN, stream=None,
                weight_mode=L.MGS_WEIGHT_EQ3):
        phi = L.ptr(self.phi) if use_mlp else None
        om = L.ptr(self.omod) if use_mlp else None
        if weight_mode == L.MGS_WEIGHT_EQ3:
            L.check(L.lib().mgs_project(L.C.byref(scene.struct), L.C.byref(cam_s), phi, om, L.MGS_TILE,
                                        alpha_min, L.C.byref(self.proj), L.stream_ptr(stream)))
        else:
            L.check(L.lib().mgs_project_weighted(L.C.byref(scene.struct), L.C.byref(cam_s), phi, om, L.MGS_TILE,
                                                 alpha_min, int(weight_mode), L.C.byref(self.proj),
                                                 L.stream_ptr(stream)))

    def enhance_project(self, scene: DeviceScene, cam_s, mlp: DeviceMLP, alpha_min=ALPHA_MIN, stream=None,
                        weight_mode=L.MGS_WEIGHT_EQ3):
        """Fused enhance + project (one read of the attributes); also fills phi / omod."""
        if scene.sh_degree != 1:
            if weight_mode != L.MGS_WEIGHT_EQ3:
                raise ValueError("SH orders other than 1 are projected with the Eq. 3 weight only")
            L.check(L.lib().mgs_enhance_project_sh(L.C.byref(scene.struct), scene.sh_degree, L.C.byref(cam_s),
                                                   L.ptr(mlp.packed), L.MGS_TILE, alpha_min, L.C.byref(self.proj),
                                                   L.ptr(self.phi), L.ptr(self.omod), L.stream_ptr(stream)))
        elif weight_mode == L.MGS_WEIGHT_EQ3:
            L.check(L.lib().mgs_enhance_project(L.C.byref(scene.struct), L.C.byref(cam_s), L.ptr(mlp.packed),
                                                L.MGS_TILE, alpha_min, L.C.byref(self.proj), L.ptr(self.phi),
                                                L.ptr(self.omod), L.stream_ptr(stream)))
        else:
            L.check(L.lib().mgs_enhance_project_weighted(
                L.C.byref(scene.struct), L.C.byref(cam_s), L.ptr(mlp.packed), L.MGS_TILE, alpha_min,
                int(weight_mode), L.C.byref(self.proj), L.ptr(self.phi), L.ptr(self.omod), L.stream_ptr(stream)))

    def project_sortfree(self, scene: DeviceScene, cam_s, sigma, beta, mlp=None, alpha_min=ALPHA_MIN, stream=None,
                         fused=True):
        """Projection with Eq. 1's weight exp(-sigma d^beta) (sigma, beta: device float32 [N]);
        with ``mlp`` its opacity head modulates o (the fused enhance + project, or with
        ``fused=False`` mgs_enhance followed by mgs_project_sortfree)."""
        if mlp is None or not fused:
            if mlp is not None:
                self.enhance(scene, cam_s, mlp, stream)
            L.check(L.lib().mgs_project_sortfree(L.C.byref(scene.struct), L.C.byref(cam_s),
                                                 L.ptr(self.omod) if mlp is not None else None, L.ptr(sigma),
                                                 L.ptr(beta), L.MGS_TILE, alpha_min, L.C.byref(self.proj),
                                                 L.stream_ptr(stream)))
        else:
            L.check(L.lib().mgs_enhance_project_sortfree(
                L.C.byref(scene.struct), L.C.byref(cam_s), L.ptr(mlp.packed), L.ptr(sigma), L.ptr(beta), L.MGS_TILE,
                alpha_min, L.C.byref(self.proj), L.ptr(self.phi), L.ptr(self.omod), L.stream_ptr(stream)))

    def enhance_project_mlp_f(self, scene: DeviceScene, cam_s, mlp: DeviceMLPF, alpha_min=ALPHA_MIN, stream=None):
        """Fused MLP_f (256-128-64) enhancement + projection; also fills phi / omod."""
        L.check(L.lib().mgs_enhance_project_mlp_f(L.C.byref(scene.struct), L.C.byref(cam_s), L.ptr(mlp.packed),
                                                  L.MGS_TILE, alpha_min, L.C.byref(self.proj), L.ptr(self.phi),
                                                  L.ptr(self.omod), L.stream_ptr(stream)))

    def enhance_project_nvq(self, q: DeviceNVQ, cam_s, mlp: DeviceMLP, alpha_min=ALPHA_MIN, stream=None):
        """Fused enhance + project reading the attributes through the NVQ codebooks."""
        L.check(L.lib().mgs_enhance_project_nvq(L.C.byref(q.struct), L.C.byref(cam_s), L.ptr(mlp.packed),
                                                L.MGS_TILE, alpha_min, L.C.byref(self.proj), L.ptr(self.phi),
                                                L.ptr(self.omod), L.stream_ptr(stream)))

    def bin(self, sorted_path=False, stream=None):
        self.ensure_capacity(self.capacity, sorted_path)
        lib = L.lib()
        fn = lib.mgs_bin_sorted if sorted_path else lib.mgs_bin
        ws = self.ws_sorted if sorted_path else self.ws
        L.check(fn(L.C.byref(self.proj), self.n, self.tiles_x, self.tiles_y, L.ptr(ws), ws.numel() * 4,
                   L.ptr(self.tile_offsets), L.ptr(self.gids), self.capacity, L.ptr(self.n_pairs),
                   L.stream_ptr(stream)))

    def tile_sort(self, stream=None):
        """mgs_tile_sort: the current (order-independent) lists sorted in place by depth, ties by
        index -- the sorted path's lists, from the two-level binning plus a per-tile sort."""
        if self.ws_tsort is None or self.ws_tsort_cap != self.capacity:
            nb = L.C.c_size_t()
            L.check(L.lib().mgs_tile_sort_workspace(self.tiles_x, self.tiles_y, self.capacity, L.C.byref(nb)))
            self.ws_tsort = torch.empty((nb.value + 255) // 256 * 64, dtype=torch.float32, device=self.device)
            self.ws_tsort_cap = self.capacity
        L.check(L.lib().mgs_tile_sort(L.C.byref(self.proj), self.n, L.ptr(self.tile_offsets), L.ptr(self.gids),
                                      self.tiles_x, self.tiles_y, self.capacity, L.ptr(self.n_pairs),
                                      L.ptr(self.ws_tsort), self.ws_tsort.numel() * 4, L.stream_ptr(stream)))

    def blend_oit(self, cam_s, bg=(0.0, 0.0, 0.0), alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, want_aux=False,
                  stream=None, split=True, w_bg=None):
        """Eq. 2 composite (Eq. 1's with a background weight ``w_bg``); ``split`` (default) uses the
        split-tile blend that balances dense tiles."""
        if want_aux and self.aux is None:
            self.aux = torch.empty(5, self.H, self.W, dtype=torch.float32, device=self.device)
        if w_bg is not None:
            aux = L.ptr(self.aux) if want_aux else None
            if split:
                L.check(L.lib().mgs_blend_sortfree_split(
                    L.C.byref(self.proj), L.ptr(self.tile_offsets), L.ptr(self.gids), L.ptr(self.n_pairs),
                    self.capacity, L.C.byref(cam_s), L.MGS_TILE, L.bg_array(bg), float(w_bg), alpha_min, alpha_max,
                    L.ptr(self.ws_split), self.ws_split.numel() * 4, L.ptr(self.image), aux, L.stream_ptr(stream)))
            else:
                L.check(L.lib().mgs_blend_sortfree(
                    L.C.byref(self.proj), L.ptr(self.tile_offsets), L.ptr(self.gids), L.C.byref(cam_s), L.MGS_TILE,
                    L.bg_array(bg), float(w_bg), alpha_min, alpha_max, L.ptr(self.image), aux, L.stream_ptr(stream)))
            return
        if split:
            L.check(L.lib().mgs_blend_oit_split(
                L.C.byref(self.proj), L.ptr(self.tile_offsets), L.ptr(self.gids), L.ptr(self.n_pairs), self.capacity,
                L.C.byref(cam_s), L.MGS_TILE, L.bg_array(bg), alpha_min, alpha_max, L.ptr(self.ws_split),
                self.ws_split.numel() * 4, L.ptr(self.image), L.ptr(self.aux) if want_aux else None,
                L.stream_ptr(stream)))
            return
        L.check(L.lib().mgs_blend_oit(L.C.byref(self.proj), L.ptr(self.tile_offsets), L.ptr(self.gids),
                                      L.C.byref(cam_s), L.MGS_TILE, L.bg_array(bg), alpha_min, alpha_max,
                                      L.ptr(self.image), L.ptr(self.aux) if want_aux else None,
                                      L.stream_ptr(stream)))

    def blend_sorted(self, cam_s, bg=(0.0, 0.0, 0.0), alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, t_stop=T_STOP,
                     stream=None):
        L.check(L.lib().mgs_blend_sorted(L.C.byref(self.proj), L.ptr(self.tile_offsets), L.ptr(self.gids),
                                         L.C.byref(cam_s), L.MGS_TILE, L.bg_array(bg), alpha_min, alpha_max,
                                         t_stop, L.ptr(self.image), L.stream_ptr(stream)))

    def pairs(self):
        return int(_u32_to_i64(self.n_pairs)[0])

    def check_capacity(self, stream=None):
        """mgs_check_capacity after a binning: waits for the stream and returns the pair count
        (above self.capacity the lists were not written)."""
        P = L.C.c_uint64()
        rc = L.lib().mgs_check_capacity(L.ptr(self.n_pairs), self.capacity, L.C.byref(P), L.stream_ptr(stream))
        if rc != L.MGS_ERR_CAPACITY:
            L.check(rc)
        return int(P.value)

    def census(self, cam_s, alpha_min=ALPHA_MIN, stream=None):
        """mgs_blend_census on the current lists: (list entries, evaluations the OIT blend
        executes, contributing pixel-Gaussian pairs); synchronises."""
        out = torch.empty(3, dtype=torch.int64, device=self.device)
        L.check(L.lib().mgs_blend_census(L.C.byref(self.proj), L.ptr(self.tile_offsets), L.ptr(self.gids),
                                         L.ptr(self.n_pairs), self.capacity, L.C.byref(cam_s), alpha_min,
                                         L.ptr(out), L.stream_ptr(stream)))
        return tuple(int(v) for v in out.cpu())

    # -- whole pass -----------------------------------------------------------
    def render(self, scene, cam, mlp=None, bg=(0.0, 0.0, 0.0), sorted_path=False, want_aux=False,
               check_capacity=True, stream=None, fused=False, split=True, weight_mode=L.MGS_WEIGHT_EQ3,
               sortfree=None, w_bg=None):
        """enhance -> project -> bin -> blend (``scene`` a DeviceScene, or a DeviceNVQ whose
        attributes are read through its codebooks).  With check_capacity the host reads the
        pair count once and re-bins with a larger capacity on overflow.  ``weight_mode``
        selects Eq. 3 or one of its ablations (MGS_WEIGHT_*); ``sortfree`` = (sigma, beta)
        device arrays with ``w_bg`` selects Eq. 1 (SortFreeGS weight and composite).  ``sorted_path``
        True sorts all pairs by (tile, depth); "tile_sort" bins as the order-independent path and
        sorts each tile's list by depth (identical lists, mgs_tile_sort)."""
        cam_s = L.make_camera(cam)
        if (sortfree is None) != (w_bg is None):
            raise ValueError("Eq. 1 needs both sortfree=(sigma, beta) and w_bg")
        if sortfree is not None:
            if sorted_path or not isinstance(scene, DeviceScene) or scene.sh_degree != 1 or isinstance(mlp, DeviceMLPF):
                raise ValueError("Eq. 1 renders float32 first-order-SH scenes on the order-independent path")
            self.project_sortfree(scene, cam_s, sortfree[0], sortfree[1], mlp=mlp, stream=stream, fused=fused)
        elif isinstance(scene, DeviceNVQ):
            if mlp is None:
                raise ValueError("a vector-quantised scene renders through the fused enhance + project (needs an MLP)")
            if weight_mode != L.MGS_WEIGHT_EQ3:
                raise ValueError("the vector-quantised path computes the Eq. 3 weight only")
            self.enhance_project_nvq(scene, cam_s, mlp, stream=stream)
        elif isinstance(mlp, DeviceMLPF):
            if weight_mode != L.MGS_WEIGHT_EQ3 or scene.sh_degree != 1:
                raise ValueError("the MLP_f path computes first-order SH and the Eq. 3 weight only")
            self.enhance_project_mlp_f(scene, cam_s, mlp, stream=stream)
        elif mlp is not None and (fused or scene.sh_degree != 1):
            self.enhance_project(scene, cam_s, mlp, stream=stream, weight_mode=weight_mode)
        else:
            if scene.sh_degree != 1:
                raise ValueError("SH orders other than 1 render through the fused enhance + project (needs an MLP)")
            if mlp is not None:
                self.enhance(scene, cam_s, mlp, stream)
            self.project(scene, cam_s, use_mlp=mlp is not None, stream=stream, weight_mode=weight_mode)
        # sorted_path: True = global (tile, depth) radix sort of the pairs; "tile_sort" = the
        # order-independent binning followed by a per-tile depth sort (the same lists)
        global_sort = bool(sorted_path) and sorted_path != "tile_sort"
        self.bin(global_sort, stream)
        if check_capacity:
            P = self.check_capacity(stream)      # synchronises
            if P > self.capacity:
                self.ensure_capacity(int(P * 1.25) + 1024, global_sort)
                self.bin(global_sort, stream)
        if sorted_path == "tile_sort":
            self.tile_sort(stream)
        if sorted_path:
            self.blend_sorted(cam_s, bg, stream=stream)
        else:
            self.blend_oit(cam_s, bg, want_aux=want_aux, stream=stream, split=split, w_bg=w_bg)
        return self.image

    # -- views for tests ---------------------------------------------------------
    def lists(self):
        P = self.pairs()
        return _u32_to_i64(self.tile_offsets).cpu(), _u32_to_i64(self.gids[:P]).cpu()

    def decoded(self):
        """Projected record as float64 numpy arrays (for stage parity checks)."""
        s = self.splat.double().cpu().numpy()
        rect = _u32_to_i64(self.rect).cpu().numpy()
        LOG2E = 1.4426950408889634
        A = s[:, 4] / (-0.5 * LOG2E)
        out = dict(mean2d=s[:, 0:2], log2o=s[:, 2], w=s[:, 3], A=A, beta=s[:, 5],
                   inv_c=s[:, 6] / (-0.5 * LOG2E), depth=s[:, 7], color=s[:, 8:11], o_eff=s[:, 11],
                   rect=np.stack([rect[:, 0] & 0xFFFF, rect[:, 0] >> 16, rect[:, 1] & 0xFFFF, rect[:, 1] >> 16], 1),
                   n_tiles=_u32_to_i64(self.n_tiles).cpu().numpy())
        return out
