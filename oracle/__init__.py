"""FP64 CPU oracle of the butterfly matched-filter hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import, call or execute anything here.  The
oracle shares no code with the HIP path and never imports it.
"""
from .bfsearch_oracle import (
    hann,
    chirp_template,
    grid_params,
    template_bank,
    correlate_fft,
    correlate_direct,
    sigma_time,
    sigma_parseval,
    sigma_eq7,
    threshold_tails,
    search,
    max_projection,
    pair_segments,
    coincidences,
    TAIL_DTYPE,
    PEAK_DTYPE,
    COINC_DTYPE,
)

__all__ = [
    "hann",
    "chirp_template",
    "grid_params",
    "template_bank",
    "correlate_fft",
    "correlate_direct",
    "sigma_time",
    "sigma_parseval",
    "sigma_eq7",
    "threshold_tails",
    "search",
    "max_projection",
    "pair_segments",
    "coincidences",
    "TAIL_DTYPE",
    "PEAK_DTYPE",
    "COINC_DTYPE",
]
