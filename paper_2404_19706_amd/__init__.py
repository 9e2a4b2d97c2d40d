"""MI355X (gfx950) masked differentiable Gaussian rasterizer: the mapping
hot path of RTG-SLAM (arXiv 2404.19706) as a C-ABI HIP library
(include/rtg.h, librtg.so) with a thin torch binding."""
from ._lib import RtgError, default_config, lib  # noqa: F401
from .rasterizer import Rasterizer, rasterize_masked  # noqa: F401

__all__ = ["Rasterizer", "rasterize_masked", "RtgError", "default_config", "lib"]
