"""MI355X-native order-independent Gaussian splatting (Mobile-GS render pass).

The numeric work lives in libmgs.so (hand-written gfx950 HIP kernels behind
the C ABI of include/mgs.h); this package is the thin Python layer over it.
"""
from . import _lib
from .render import ALPHA_MAX, ALPHA_MIN, T_STOP, DeviceMLP, DeviceMLPF, DeviceNVQ, DeviceScene, Renderer

__all__ = ["DeviceScene", "DeviceNVQ", "DeviceMLP", "DeviceMLPF", "Renderer", "ALPHA_MIN", "ALPHA_MAX", "T_STOP", "_lib"]
