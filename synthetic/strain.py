"""Band-limited Gaussian strain with chirp injections (seeded, FP64).

Stand-in for the paper's data base (Sec. 2): LIGO S6 H1/L1 strain sampled at
4096 Hz and band-passed to 350-2000 Hz, where the noise is close to Gaussian.
The real frames are not available here; these generators reproduce the
shape (sample rate, band, segment length) and the Gaussian statistics, not
instrumental lines.

Seeds: ``numpy.random.SeedSequence(entropy=170801609,
spawn_key=(config_id, channel, segment_idx, purpose))`` with PCG64, where
purpose is one of ``noise``, ``inject_params``, ``offsets``, ``arrivals``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ENTROPY = 170801609
_PURPOSE = {"noise": 0, "inject_params": 1, "offsets": 2, "arrivals": 3, "lengths": 4}


def seeded_rng(config_id: int, channel: int, segment_idx: int, purpose: str) -> np.random.Generator:
    """PCG64 generator for one (config, channel, segment, purpose) stream."""
    ss = np.random.SeedSequence(
        entropy=ENTROPY, spawn_key=(int(config_id), int(channel), int(segment_idx), _PURPOSE[purpose])
    )
    return np.random.Generator(np.random.PCG64(ss))


def bandlimited_noise(n: int, fs: float, rng: np.random.Generator,
                      band: tuple[float, float] = (350.0, 2000.0)) -> np.ndarray:
    """White N(0,1) FP64 noise passed through an FFT brick-wall band-pass.

    Bins with band[0] <= k*fs/n <= band[1] are kept (edges inclusive); DC and
    Nyquist are always zeroed.  The result is real FP64 of length n.
    """
    x = rng.standard_normal(n)
    spec = np.fft.rfft(x)
    freqs = np.arange(n // 2 + 1, dtype=np.float64) * (fs / n)
    keep = (freqs >= band[0]) & (freqs <= band[1])
    keep[0] = False
    keep[-1] = False
    spec[~keep] = 0.0
    return np.fft.irfft(spec, n=n)


def unit_hann_chirp(f0: float, fdot: float, length: int, fs: float) -> np.ndarray:
    """Hann-tapered linear chirp of unit energy, used as an injected signal.

    Instantaneous frequency f0 + fdot*t over t = m/fs, m < length; the taper is
    the symmetric Hann window 0.5*(1 - cos(2*pi*m/(length-1))).
    """
    m = np.arange(length, dtype=np.float64)
    t = m / fs
    cycles = f0 * t + 0.5 * fdot * t * t
    taper = 0.5 - 0.5 * np.cos(2.0 * np.pi * m / (length - 1)) if length > 1 else np.ones(1)
    s = taper * np.cos(2.0 * np.pi * (cycles - np.floor(cycles)))
    return s / np.sqrt(np.dot(s, s))


@dataclass(frozen=True)
class Injection:
    """One injected chirp: parameters, amplitude (= matched-filter SNR) and sample offset."""

    f0: float
    fdot: float
    tau: float
    snr: float
    offset: int

    def waveform(self, fs: float) -> np.ndarray:
        length = int(round(self.tau * fs))
        return self.snr * unit_hann_chirp(self.f0, self.fdot, length, fs)


def add_injections(y: np.ndarray, injections: list[Injection], fs: float) -> np.ndarray:
    """Add injections to y (after the band-pass) at their offsets; returns a new array."""
    out = y.copy()
    for inj in injections:
        w = inj.waveform(fs)
        out[inj.offset:inj.offset + len(w)] += w
    return out


def draw_injections(rng_params: np.random.Generator, rng_offsets: np.random.Generator,
                    count: int, n: int, fs: float, tau: float,
                    f0_range: tuple[float, float], fdot_range: tuple[float, float],
                    snr_range: tuple[float, float],
                    inband: tuple[float, float] = (400.0, 1900.0)) -> list[Injection]:
    """Draw `count` non-overlapping in-band chirp injections.

    f0 and fdot are uniform on their ranges, redrawn until the frequency stays
    within `inband` over the chirp; SNR is uniform on snr_range; offsets are
    uniform integers in [0, n - L] and are redrawn until no two chirps overlap.
    """
    length = int(round(tau * fs))
    params = []
    while len(params) < count:
        f0 = rng_params.uniform(*f0_range)
        fdot = rng_params.uniform(*fdot_range)
        f_end = f0 + fdot * tau
        if not (inband[0] <= f0 <= inband[1] and inband[0] <= f_end <= inband[1]):
            continue
        snr = rng_params.uniform(*snr_range)
        params.append((f0, fdot, snr))
    offsets: list[int] = []
    tries = 0
    while len(offsets) < count:
        tries += 1
        if tries > 100000:
            raise RuntimeError("cannot place non-overlapping injections")
        o = int(rng_offsets.integers(0, n - length + 1))
        if all(abs(o - p) >= length for p in offsets):
            offsets.append(o)
    return [Injection(f0, fdot, tau, snr, off) for (f0, fdot, snr), off in zip(params, offsets)]
