"""The five benchmark workloads (segment shapes, template grids, thresholds).

Each workload names the synthetic segments it draws and the chirp grid it
searches.  Template id = i_f0 * n_fdot + i_fdot (f0-major), with
f0 = linspace(f0_lo, f0_hi, n_f0) and fdot = linspace(fdot_lo, fdot_hi,
n_fdot), both inclusive; template j has duration taus[j % len(taus)].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .strain import (
    Injection,
    add_injections,
    bandlimited_noise,
    draw_injections,
    seeded_rng,
)


@dataclass(frozen=True)
class Workload:
    name: str
    config_id: int
    n: int                                  # segment length (max length for uneven workloads)
    fs: float
    n_segments: int
    n_f0: int
    n_fdot: int
    f0_range: tuple[float, float]
    fdot_range: tuple[float, float]
    taus: tuple[float, ...]
    kappa: float
    dtype: str                              # "f64" or "f32" sample precision
    lengths: tuple[int, ...] = ()           # uneven workloads: allowed segment lengths
    injections_per_segment: tuple[int, int] = (0, 0)
    snr_range: tuple[float, float] = (8.0, 15.0)
    fixed_injection: tuple[float, float, float, float] | None = None  # (f0, fdot, tau, snr)
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_templates(self) -> int:
        return self.n_f0 * self.n_fdot

    def template_params(self) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(f0, fdot, tau) per template id, FP64."""
        f0s = np.linspace(self.f0_range[0], self.f0_range[1], self.n_f0)
        fds = np.linspace(self.fdot_range[0], self.fdot_range[1], self.n_fdot)
        j = np.arange(self.n_templates)
        taus = np.asarray(self.taus, dtype=np.float64)
        return f0s[j // self.n_fdot], fds[j % self.n_fdot], taus[j % len(taus)]


WORKLOADS: dict[str, Workload] = {
    "C1": Workload(
        name="C1", config_id=1, n=1 << 13, fs=4096.0, n_segments=1,
        n_f0=8, n_fdot=8, f0_range=(400.0, 1800.0), fdot_range=(-200.0, 200.0),
        taus=(0.25,), kappa=4.0, dtype="f64",
        fixed_injection=(600.0, 50.0, 0.25, 20.0),
        description="plain method, FP64: N=2^13, 64 chirps of 1024 samples, one SNR-20 injection, kappa=4",
    ),
    "C2": Workload(
        name="C2", config_id=2, n=1 << 16, fs=4096.0, n_segments=1,
        n_f0=128, n_fdot=64, f0_range=(350.0, 2000.0), fdot_range=(-500.0, 500.0),
        taus=(1.0,), kappa=5.0, dtype="f32", injections_per_segment=(3, 3), snr_range=(8.0, 15.0),
        description="paper shape, FP32: N=2^16, 8192 one-second chirps (128 f0 x 64 fdot), 3 injections, kappa=5",
    ),
    "C3": Workload(
        name="C3", config_id=2, n=1 << 16, fs=4096.0, n_segments=1,
        n_f0=1024, n_fdot=1024, f0_range=(350.0, 2000.0), fdot_range=(-500.0, 500.0),
        taus=(1.0,), kappa=5.5, dtype="f32", injections_per_segment=(3, 3), snr_range=(8.0, 15.0),
        description="full dense bank: the C2 segment against 1024 x 1024 one-second chirps, kappa=5.5",
    ),
    "C4": Workload(
        name="C4", config_id=4, n=1 << 17, fs=4096.0, n_segments=64,
        n_f0=256, n_fdot=256, f0_range=(350.0, 2000.0), fdot_range=(-500.0, 500.0),
        taus=(0.5, 1.0, 2.0), kappa=5.0, dtype="f32",
        lengths=(1 << 14, 1 << 15, 1 << 16, 1 << 17), injections_per_segment=(0, 2), snr_range=(8.0, 15.0),
        description="batched uneven: 64 segments of 2^14..2^17 samples, 65536 chirps with tau in {0.5,1,2} s",
    ),
    "C5": Workload(
        name="C5", config_id=5, n=1 << 17, fs=4096.0, n_segments=0,
        n_f0=512, n_fdot=512, f0_range=(350.0, 2000.0), fdot_range=(-500.0, 500.0),
        taus=(1.0,), kappa=5.0, dtype="f32",
        lengths=(1 << 14, 1 << 15, 1 << 16, 1 << 17), snr_range=(6.0, 20.0),
        description="served stream: Poisson arrivals at 8/s from 4 channels, 262144 chirps, FP16 spectra",
        extra={"rate_hz": 8.0, "channels": 4, "inject_rate": 0.01, "duration_s": 600.0},
    ),
}


def get_workload(name: str) -> Workload:
    return WORKLOADS[name]


def segment_length(w: Workload, segment_idx: int, channel: int = 0) -> int:
    if not w.lengths:
        return w.n
    r = seeded_rng(w.config_id, channel, segment_idx, "lengths")
    return int(w.lengths[int(r.integers(0, len(w.lengths)))])


def make_segment(w: Workload, segment_idx: int = 0, channel: int = 0) -> tuple[np.ndarray, list[Injection]]:
    """One synthetic segment of workload w: FP64 samples and the injections it carries.

    The samples are returned in FP64; FP32 workloads cast them with
    ``astype(np.float32)`` and both the oracle and the GPU path consume the
    cast values.
    """
    n = segment_length(w, segment_idx, channel)
    y = bandlimited_noise(n, w.fs, seeded_rng(w.config_id, channel, segment_idx, "noise"))
    r_par = seeded_rng(w.config_id, channel, segment_idx, "inject_params")
    r_off = seeded_rng(w.config_id, channel, segment_idx, "offsets")
    if w.fixed_injection is not None:
        f0, fdot, tau, snr = w.fixed_injection
        length = int(round(tau * w.fs))
        off = int(r_off.integers(0, n - length + 1))
        injections = [Injection(f0, fdot, tau, snr, off)]
    else:
        lo, hi = w.injections_per_segment
        count = int(r_par.integers(lo, hi + 1)) if hi > lo else lo
        tau = 1.0 if 1.0 in w.taus else w.taus[0]
        injections = draw_injections(r_par, r_off, count, n, w.fs, tau,
                                     w.f0_range, w.fdot_range, w.snr_range) if count else []
    y = add_injections(y, injections, w.fs)
    if w.dtype == "f32":
        y = y.astype(np.float32)
    return y, injections


def make_pair(w: Workload, segment_idx: int = 0) -> tuple[np.ndarray, np.ndarray, list[Injection]]:
    """Two time-aligned detector channels of one segment of workload w: channel 0 is
    make_segment(w, segment_idx); channel 1 carries independent band-limited noise (its own
    seed) plus the same injections at the same offsets, as a signal seen by both detectors."""
    a, injections = make_segment(w, segment_idx, channel=0)
    b = bandlimited_noise(len(a), w.fs, seeded_rng(w.config_id, 1, segment_idx, "noise"))
    b = add_injections(b, injections, w.fs)
    if w.dtype == "f32":
        b = b.astype(np.float32)
    return a, b, injections


def make_segments(w: Workload, count: int | None = None, channel: int = 0):
    """List of (samples, injections) for segments 0..count-1 of workload w."""
    count = w.n_segments if count is None else count
    return [make_segment(w, i, channel) for i in range(count)]


@dataclass(frozen=True)
class Arrival:
    """One request of a served stream: when it arrives, from which channel, its length."""

    index: int
    time: float        # seconds since the start of the stream
    channel: int
    length: int
    inject: bool       # carries one chirp injection


def arrivals(w: Workload, duration_s: float | None = None) -> list[Arrival]:
    """Poisson arrivals at w.extra['rate_hz'] (all channels together) over duration_s
    (default w.extra['duration_s']); channel and length uniform, an injection with probability
    w.extra['inject_rate'].  A shorter duration gives a prefix of a longer one."""
    rate, channels = float(w.extra["rate_hz"]), int(w.extra["channels"])
    p_inj = float(w.extra.get("inject_rate", 0.0))
    dur = float(w.extra["duration_s"] if duration_s is None else duration_s)
    r = seeded_rng(w.config_id, 0, 0, "arrivals")
    out: list[Arrival] = []
    t = 0.0
    while True:
        t += float(r.exponential(1.0 / rate))
        if t >= dur:
            return out
        ch = int(r.integers(0, channels))
        n = int(w.lengths[int(r.integers(0, len(w.lengths)))])
        inj = bool(r.random() < p_inj)
        out.append(Arrival(len(out), t, ch, n, inj))


def request_samples(w: Workload, a: Arrival) -> tuple[np.ndarray, list[Injection]]:
    """Samples of one served request (seeded by its channel and index) and its injections."""
    y = bandlimited_noise(a.length, w.fs, seeded_rng(w.config_id, a.channel, a.index, "noise"))
    injections: list[Injection] = []
    if a.inject:
        tau = 1.0 if 1.0 in w.taus else w.taus[0]
        injections = draw_injections(seeded_rng(w.config_id, a.channel, a.index, "inject_params"),
                                     seeded_rng(w.config_id, a.channel, a.index, "offsets"),
                                     1, a.length, w.fs, tau, w.f0_range, w.fdot_range, w.snr_range)
        y = add_injections(y, injections, w.fs)
    if w.dtype == "f32":
        y = y.astype(np.float32)
    return y, injections
