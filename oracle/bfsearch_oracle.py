"""Plain FP64 oracle of butterfly matched filtering (arXiv:1708.01609, Sec. 3).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and
bench.py's cpu_baseline leg, never by the product path.  No code is shared
with the HIP library.

What it computes, per segment y (length N) and template w (length L <= N):

* rho[n] = sum_{m<L} w[m] * y[(n + m) mod N], n = 0..N-1 -- the discrete,
  circular form of the correlation integral Eq. (3).  It is circular because
  the template is zero-padded to N and correlated by length-N FFTs
  (Sec. 3.2, step (ii)); the integrand's "dt" is read as ds.
* evaluated by the three-step FFT correlation Eq. (5): forward real FFTs of
  the zero-padded template and of the segment, the product conj(W)*Y (the
  correlation theorem stated before Eq. (4)), and an inverse FFT, all in FP64
  with scipy.fft.  For tiny N the direct sum above is available as well.
* sigma = sqrt(sum_n rho[n]^2 / N), the RMS about zero of Eq. (6) (both y and
  w are taken to have vanishing mean, as the paper states).
* its Parseval form.  With unnormalised C_k = sum_n rho[n] exp(-2 pi i k n/N),
  sigma = (1/N) sqrt(|C_0|^2 + |C_{N/2}|^2 + 2 sum_{k=1}^{N/2-1} |C_k|^2).
  The paper's Eq. (7) (sqrt(2)/N times the sum over k=1..N/2-1) equals this
  exactly when C_0 = C_{N/2} = 0, i.e. for band-limited data; the 1/N on the
  forward transform in Eq. (8) is inconsistent with Eq. (7) and is read as
  a typo (see sigma_eq7).
* tails: every (segment, template, lag) with |rho| > kappa * sigma, Eq. (9)
  applied to the absolute value as the text after it says; strict '>'.
  This is the "gather all hits" mode of Sec. 3.3 (no max selection).
* the per-lag max projection of Sec. 3.3 (Eqs. 13-17): over all templates,
  for every (segment, lag) that carries a tail, the tail of largest
  significance |rho| / sigma (the quantity the threshold compares), reported
  as the signed rho / sigma with its template.  The paper's update of the
  projection array is racy (its text says so); here equal significances go to
  the lowest template id, so the result is unique (see max_projection).
* two detectors (Sec. 3.2 step (i) processes H1 and L1 segments as pairs;
  Sec. 5 and Table 3): the two channels of a pair are time-aligned segments
  of equal length, searched like any other segment (pair p's channels are
  segments 2p and 2p + 1).  A coincidence is a lag at which both channels
  carry a projected hit and the initial frequencies of the two winning
  templates differ by less than Delta (the "simultaneous hits with frequency
  pairs within Delta = 50 Hz" of Sec. 5), see coincidences.

Templates (Sec. 2 uses chirps from a spin-down model that the paper does not
give; linear chirps stand in): w[m] = h[m] cos(2 pi (f0 t + fdot t^2 / 2)),
t = m / fs, with h the symmetric Hann window, normalised to sum w^2 = 1.
The phase is reduced modulo one cycle before the cosine.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

TAIL_DTYPE = np.dtype([("segment", np.uint32), ("template", np.uint32), ("lag", np.uint32), ("rho", np.float64)])
PEAK_DTYPE = np.dtype([("segment", np.uint32), ("lag", np.uint32), ("template", np.uint32), ("snr", np.float64)])
COINC_DTYPE = np.dtype([("pair", np.uint32), ("lag", np.uint32), ("template_a", np.uint32), ("template_b", np.uint32),
                        ("snr_a", np.float64), ("snr_b", np.float64)])


def _workers() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


# ---------------------------------------------------------------- templates --

def hann(length: int) -> np.ndarray:
    """Symmetric Hann window h[m] = (1 - cos(2 pi m / (L-1))) / 2, m = 0..L-1 (L=1 gives [1])."""
    if length == 1:
        return np.ones(1)
    m = np.arange(length, dtype=np.float64)
    return 0.5 * (1.0 - np.cos(2.0 * np.pi * m / (length - 1)))


def chirp_template(f0: float, fdot: float, length: int, fs: float,
                   taper: bool = True, normalize: bool = True, symmetric: bool = False) -> np.ndarray:
    """Linear chirp template, FP64: h[m] cos(2 pi frac(f0 t + fdot t^2 / 2)), t = m/fs.

    Stand-in for the time-sliced spin-down chirps of Sec. 2; f0 is the
    initial frequency (the quantity Table 3 lists per hit).  Sampled as
    written, aliasing included; unit energy when normalize is set.
    symmetric: the time-symmetric template of the paper's banks (Fig. 2
    caption), the chirp plus its own time reversal, x[m] + x[L-1-m], which
    matches ascending and descending chirps alike; normalised after the sum.
    """
    t = np.arange(length, dtype=np.float64) / fs
    cycles = f0 * t + 0.5 * fdot * t * t
    w = np.cos(2.0 * np.pi * (cycles - np.floor(cycles)))
    if taper:
        w = w * hann(length)
    if symmetric:
        w = w + w[::-1]
    if normalize:
        e = np.dot(w, w)
        if e > 0:
            w = w / np.sqrt(e)
    return w


def grid_params(n_f0: int, n_fdot: int, f0_range, fdot_range, taus) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(f0, fdot, tau) per template id j = i_f0 * n_fdot + i_fdot over inclusive linspace grids."""
    f0s = np.linspace(float(f0_range[0]), float(f0_range[1]), int(n_f0))
    fds = np.linspace(float(fdot_range[0]), float(fdot_range[1]), int(n_fdot))
    taus = np.atleast_1d(np.asarray(taus, dtype=np.float64))
    j = np.arange(int(n_f0) * int(n_fdot))
    return f0s[j // int(n_fdot)], fds[j % int(n_fdot)], taus[j % len(taus)]


def template_bank(f0: np.ndarray, fdot: np.ndarray, tau: np.ndarray, fs: float,
                  taper: bool = True, ids=None, symmetric: bool = False) -> list[np.ndarray]:
    """Unit-energy chirps for the selected template ids (all when ids is None)."""
    ids = range(len(f0)) if ids is None else ids
    return [chirp_template(f0[j], fdot[j], int(round(tau[j] * fs)), fs, taper=taper, symmetric=symmetric)
            for j in ids]


# -------------------------------------------------------------- correlation --

def correlate_fft(y: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Circular correlation rho[n] = sum_m w[m] y[(n+m) mod N] by Eq. (5), FP64.

    w may be a single template (1-D) or a stack [K, L]; L <= N = len(y).
    """
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[-1]
    w = np.asarray(w, dtype=np.float64)
    if w.shape[-1] > n:
        raise ValueError("template longer than segment")
    wt = sfft.rfft(w, n=n, axis=-1, workers=_workers())
    yt = sfft.rfft(y, workers=_workers())
    return sfft.irfft(np.conj(wt) * yt, n=n, axis=-1, workers=_workers())


def correlate_direct(y: np.ndarray, w: np.ndarray) -> np.ndarray:
    """The same circular correlation as a direct O(N L) sum (Eq. (3) discretised), FP64."""
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = y.shape[0]
    rho = np.zeros(n)
    for m in range(w.shape[0]):
        rho += w[m] * np.roll(y, -m)
    return rho


# --------------------------------------------------------------------- sigma --

def sigma_time(rho: np.ndarray) -> np.ndarray:
    """Eq. (6): sqrt(sum_n rho_n^2 / N) along the last axis."""
    rho = np.asarray(rho, dtype=np.float64)
    return np.sqrt(np.sum(rho * rho, axis=-1) / rho.shape[-1])


def sigma_parseval(c_half: np.ndarray, n: int) -> np.ndarray:
    """Parseval form of Eq. (6) from the half spectrum C_0..C_{N/2} of rho (unnormalised DFT).

    sigma = (1/N) sqrt(|C_0|^2 + |C_{N/2}|^2 + 2 sum_{k=1}^{N/2-1} |C_k|^2); exact
    for any real rho of even length N.
    """
    p = np.abs(np.asarray(c_half)) ** 2
    s = p[..., 0] + p[..., n // 2] + 2.0 * np.sum(p[..., 1:n // 2], axis=-1)
    return np.sqrt(s) / n


def sigma_eq7(c_half: np.ndarray, n: int) -> np.ndarray:
    """Eq. (7) as printed, sqrt(2)/N * sqrt(sum_{k=1}^{N/2-1} |C_k|^2), with unnormalised C_k.

    Equal to sigma_parseval when C_0 = C_{N/2} = 0 (band-limited data).
    """
    p = np.abs(np.asarray(c_half)) ** 2
    return np.sqrt(2.0) / n * np.sqrt(np.sum(p[..., 1:n // 2], axis=-1))


# --------------------------------------------------------------------- tails --

def threshold_tails(rho: np.ndarray, sigma: float, kappa: float, kappa_hi: float = 0.0) -> np.ndarray:
    """Lags n with |rho_n| > kappa * sigma (Eq. (9) on the absolute value), ascending.

    kappa_hi > 0 keeps a finite band instead, kappa sigma < |rho_n| < kappa_hi sigma: the
    generalisation the paper proposes for very deep searches (Sec. 5)."""
    if not sigma > 0:
        return np.zeros(0, dtype=np.int64)
    keep = np.abs(rho) > kappa * sigma
    if kappa_hi > 0:
        keep &= np.abs(rho) < kappa_hi * sigma
    return np.nonzero(keep)[0]


def search(segments, templates, kappa: float, keep_rho: bool = False, chunk: int = 128, kappa_hi: float = 0.0):
    """Full oracle: every segment against every template.

    segments: list of 1-D arrays (FP32 inputs are upcast exactly to FP64).
    templates: list of 1-D FP64 templates (lengths may differ, each <= its segment).
    Returns dict with 'sigma' [S, K] (Eq. (6), time domain), 'sigma_f' [S, K]
    (Parseval form), 'tails' (TAIL_DTYPE, sorted by segment, template, lag)
    and, with keep_rho, 'rho' as a list over segments of [K, N_s] arrays.
    """
    n_seg, n_tmp = len(segments), len(templates)
    sig = np.zeros((n_seg, n_tmp))
    sig_f = np.zeros((n_seg, n_tmp))
    tails = []
    rhos = []
    for s, y in enumerate(segments):
        y = np.asarray(y).astype(np.float64)
        n = y.shape[0]
        yt = sfft.rfft(y, workers=_workers())
        rho_s = np.zeros((n_tmp, n)) if keep_rho else None
        # group templates of equal length so each group is one batched transform
        for j0 in range(0, n_tmp, chunk):
            js = list(range(j0, min(n_tmp, j0 + chunk)))
            wmat = np.zeros((len(js), n))
            for r, j in enumerate(js):
                w = np.asarray(templates[j], dtype=np.float64)
                if w.shape[0] > n:
                    raise ValueError("template longer than segment")
                wmat[r, :w.shape[0]] = w
            c = np.conj(sfft.rfft(wmat, axis=-1, workers=_workers())) * yt
            rho = sfft.irfft(c, n=n, axis=-1, workers=_workers())
            sg = sigma_time(rho)
            sig[s, js] = sg
            sig_f[s, js] = sigma_parseval(c, n)
            for r, j in enumerate(js):
                lags = threshold_tails(rho[r], sg[r], kappa, kappa_hi)
                if lags.size:
                    t = np.zeros(lags.size, dtype=TAIL_DTYPE)
                    t["segment"] = s
                    t["template"] = j
                    t["lag"] = lags
                    t["rho"] = rho[r, lags]
                    tails.append(t)
            if keep_rho:
                rho_s[js] = rho
        if keep_rho:
            rhos.append(rho_s)
    tails = np.concatenate(tails) if tails else np.zeros(0, dtype=TAIL_DTYPE)
    tails = np.sort(tails, order=("segment", "template", "lag"))
    out = {"sigma": sig, "sigma_f": sig_f, "tails": tails}
    if keep_rho:
        out["rho"] = rhos
    return out


def max_projection(tails: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """Per-lag max projection of a tail list (Sec. 3.3, Eqs. 13-17).

    tails: TAIL_DTYPE records; sigma: [S, K] sigma of every correlation.  For each
    (segment, lag) present in `tails`, keep the tail with the largest |rho| / sigma;
    ties go to the lowest template id.  Returns PEAK_DTYPE records sorted by
    (segment, lag), with snr = rho / sigma of the kept tail (sign of rho kept).
    """
    best: dict = {}
    for s, j, n, r in zip(tails["segment"], tails["template"], tails["lag"], tails["rho"]):
        s, j, n, r = int(s), int(j), int(n), float(r)
        v = abs(r) / float(sigma[s, j])
        key = (s, n)
        if key not in best:
            best[key] = (v, j, r)
            continue
        bv, bj, _ = best[key]
        if v > bv or (v == bv and j < bj):
            best[key] = (v, j, r)
    out = np.zeros(len(best), dtype=PEAK_DTYPE)
    for i, ((s, n), (v, j, r)) in enumerate(sorted(best.items())):
        out[i] = (s, n, j, r / float(sigma[s, j]))
    return out


# -------------------------------------------------------------- two detectors --

def pair_segments(first, second):
    """Interleave the channels of detector pairs: pair p's first channel becomes segment 2p, its
    second channel segment 2p + 1 (equal lengths within a pair, Sec. 3.2 step (i))."""
    if len(first) != len(second):
        raise ValueError("every pair needs both channels")
    out = []
    for a, b in zip(first, second):
        if len(a) != len(b):
            raise ValueError("the channels of a pair must have equal lengths")
        out += [a, b]
    return out


def coincidences(proj: np.ndarray, f0: np.ndarray, delta: float) -> np.ndarray:
    """Simultaneous hits of detector pairs with close template frequencies (Sec. 5, Table 3).

    proj: PEAK_DTYPE per-lag max projection over interleaved pair segments (max_projection of
    the tails of pair_segments(...)); f0: initial frequency (Hz) of every template, which is the
    frequency the output table lists per hit; delta: Hz.  Pair p has a coincidence at lag n
    when both its channels (segments 2p, 2p + 1) carry a projected hit at n and the winning
    templates' initial frequencies satisfy |f_a - f_b| < delta.  Returns COINC_DTYPE records
    sorted by (pair, lag), with each channel's template and signed rho / sigma.
    """
    f0 = np.asarray(f0, dtype=np.float64)
    first, second = {}, {}
    for s, n, j, v in zip(proj["segment"], proj["lag"], proj["template"], proj["snr"]):
        (first if int(s) % 2 == 0 else second)[(int(s) // 2, int(n))] = (int(j), float(v))
    rows = []
    for key in sorted(first.keys() & second.keys()):
        ja, va = first[key]
        jb, vb = second[key]
        if abs(f0[ja] - f0[jb]) < delta:
            rows.append((key[0], key[1], ja, jb, va, vb))
    return np.array(rows, dtype=COINC_DTYPE) if rows else np.zeros(0, dtype=COINC_DTYPE)
