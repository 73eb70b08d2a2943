"""Seeded synthetic inputs for 2D Marchenko redatuming.

This package builds the reflection response R (in the frequency domain), the
direct arrivals G_d and the first-arrival sample indices for flat and dipping
layered earth models.  It is the one module both the FP64 oracle and the HIP
path read their inputs from; it holds none of the Marchenko method's own
arithmetic (no synthesis, mute, time reversal or series accumulation).
"""

from .layered import (  # noqa: F401
    Geometry,
    LayerModel,
    Dip,
    Problem,
    ricker_spectrum,
    random_layer_model,
    make_problem,
    make_config,
    CONFIGS,
)
