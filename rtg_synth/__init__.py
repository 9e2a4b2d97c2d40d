"""Seeded synthetic inputs: Gaussian scenes, camera poses, pixel masks and
upstream gradients.  Holds scene construction only -- none of the
rasterizer's arithmetic -- so the oracle and the HIP path can both be fed
from it."""
from .scenes import (  # noqa: F401
    CONFIGS,
    camera,
    look_at,
    make_config,
    random_upstream,
    jitter_means,
)
