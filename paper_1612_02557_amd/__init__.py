"""MI355X (gfx950) MSD radix sort of fixed-size records after RADULS
(arXiv 1612.02557): HIP kernels behind a C interface (``include/raduls.h``),
bound here with ctypes."""
from . import raduls  # noqa: F401
from .raduls import (  # noqa: F401
    sort,
    sort_segmented,
    partition,
    set_scheduler,
    load_model,
    set_tuning,
    default_tuning,
)
