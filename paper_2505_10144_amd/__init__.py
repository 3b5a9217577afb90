"""MI355X-native (gfx950) foveated Gaussian-splat rasterizer of VRSplat
(arXiv 2505.10144): Optimal-Projection preprocessing, tangent-plane tile
culling, tile|depth radix sort and single-launch foveated blending with
per-sample resorting, all in hand-written HIP kernels behind the C ABI of
include/vrs.h.  Importing the package loads nothing; the HIP library is loaded
on first use and its absence is an error (there is no other compute path)."""

__all__ = ["Renderer", "Gaussians", "upload", "rasterize", "build", "lib"]


def __getattr__(name):
    if name in ("Renderer", "Gaussians", "upload"):
        from . import render
        return getattr(render, name)
    if name == "rasterize":
        from .autograd import rasterize
        return rasterize
    if name == "build":
        from .build import build
        return build
    if name == "lib":
        from . import _lib
        return _lib
    raise AttributeError(name)
