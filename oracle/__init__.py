"""Plain FP64 CPU oracle of the HistRetinex per-image pipeline.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
calls it, and it shares no code with the GPU library.
"""

from .histretinex import (  # noqa: F401
    GRAD_OPERATORS,
    GRAD_RESCALES,
    UPDATES,
    INIT_L,
    Params,
    value_channel,
    count_histogram,
    gradient_magnitude,
    gradient_histogram,
    location_vector,
    classify,
    classify_enhanced,
    init_state,
    weights,
    update_step,
    objective,
    solve,
    target_histogram,
    matching_lut,
    equalization_lut,
    remap,
    enhance,
)
