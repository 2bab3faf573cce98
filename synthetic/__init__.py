"""Seeded synthetic low-light RGB images.

This package only draws pixels. It contains none of the enhancement method's
arithmetic, so the CPU oracle and the GPU path can both be fed from it without
sharing any of the method's code.
"""

from .lowlight import (  # noqa: F401
    BASE_SEED,
    make_image,
    make_batch_shapes,
    config_seed,
    edge_images,
)
