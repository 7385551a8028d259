"""MI355X-native SAR Differentiable Gaussian Rasterizer (SAR-GS, arXiv
2506.21633, Sec. II): HIP kernels behind a C ABI (include/sdgr.h), a thin
ctypes binding and a torch.autograd.Function.

Submodules:
  scenes  seeded synthetic scenes and radar views (inputs only)
  api     Renderer / render / SDGRFunction (loads libsdgr.so on first use)
  serve   continuous-batching render server
  train   reconstruction loop (Adam, densify/prune) and evaluation metrics
  build   compiles libsdgr.so for gfx950
"""
__version__ = "0.1.0"


def __getattr__(name):
    if name in ("RenderOptions", "GaussianTensors", "Renderer", "ForwardResult",
                "render", "SDGRFunction"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
