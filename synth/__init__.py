"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds only input generation (random numbers and how they become
record bytes); it contains none of the sorting method's arithmetic.  Every
value is a pure function of (seed, stream, index), so any index range can be
regenerated on its own, on the host (``gen``) or on the device (``device``).
"""
from .gen import (  # noqa: F401
    Spec,
    generate,
    segment_sizes,
    segment_offsets,
    segment_dists,
    zipf_cdf,
    splitmix64,
    uniform_u64,
    STREAMS,
)
