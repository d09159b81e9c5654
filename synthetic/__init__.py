"""Seeded synthetic inputs for the matched-filter hot path.

This package generates input data only: band-limited Gaussian strain segments
with chirp injections, and the workload definitions (segment lengths, template
grids, thresholds) of the five benchmark configurations.  It holds none of the
matched filter's arithmetic; both the FP64 oracle and the HIP path consume
what it produces.
"""
from .strain import (
    ENTROPY,
    seeded_rng,
    bandlimited_noise,
    unit_hann_chirp,
    Injection,
)
from .workloads import (Arrival, Workload, WORKLOADS, arrivals, get_workload, make_pair, make_segment,
                        make_segments, request_samples)

__all__ = [
    "ENTROPY",
    "seeded_rng",
    "bandlimited_noise",
    "unit_hann_chirp",
    "Injection",
    "Workload",
    "WORKLOADS",
    "get_workload",
    "make_segment",
    "make_pair",
    "make_segments",
    "Arrival",
    "arrivals",
    "request_samples",
]
