"""Helpers for GPU-vs-oracle parity checks (tolerances in units of the oracle's sigma)."""
from __future__ import annotations

import numpy as np

# Tolerances on |rho_gpu - rho_oracle| / sigma_oracle and on the tail band: FP64 path 1e-9,
# FP32 path 1e-4, 16-bit-stored template spectra 2e-3 (FP16 and BF16 alike: BF16's 8-bit
# mantissa is predicted to miss it, and the test of that form says so instead of widening it).
TOL = {"f64": 1e-9, "f32": 1e-4, "f32-w16f": 2e-3, "f32-w16b": 2e-3}

# Predicted worst error of BF16-stored spectra over 2^16 lags: rounding to an 8-bit mantissa
# gives each spectrum bin a relative error uniform in +-2^-9, so the rho error has standard
# deviation ~ 2^-8 / sqrt(3) sigma ~ 2.3e-3 sigma and its maximum over 2^16 Gaussian lags lies
# near 4.5 standard deviations (1e-2 sigma); 1.5e-2 leaves room for the tail of that maximum.
BF16_MODEL_BOUND = 1.5e-2

# A template whose sigma is below RELAX * sigma_floor lies almost wholly outside the data band.
# Finite-precision FFT error follows the input scale sigma_floor (measured FP32: ~2e-6 of it),
# not sigma, so for such a template 1e-4 sigma can sit below the rounding of the inputs.  Every
# correlation with sigma >= RELAX * floor is held to tol * sigma exactly; below that the
# tolerance scale is RELAX * floor (tol * 0.1 * floor = 1e-5 floor for FP32, 5x the measured
# error).  On the C2 bank 138 of 8192 templates fall below the cut.
RELAX = 0.1


def tol_scale(sigma, floor=None):
    """Scale that multiplies a tolerance: sigma, or RELAX * floor where sigma is smaller."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if floor is None:
        return sigma
    return np.maximum(sigma, RELAX * np.asarray(floor, dtype=np.float64))


def relaxed_mask(sigma, floor):
    """True where the relaxed scale applies (sigma < RELAX * floor)."""
    return np.asarray(sigma) < RELAX * np.asarray(floor)


def compare_tails(gpu, orc, sigma_o, kappa, tol, oracle_rho, floor=None):
    """Tail sets must agree outside a +-tol*scale band around kappa*sigma (scale = tol_scale).

    gpu: records with segment/template/lag/rho; orc: oracle TAIL_DTYPE records;
    sigma_o: [S, K] oracle sigma; oracle_rho(s, j) -> oracle rho row (for GPU
    tails the oracle did not report); floor: optional [S, K] sigma_floor values.
    Returns (n_common, n_band_only).
    """
    sc = tol_scale(sigma_o, floor)
    g = {(int(a), int(b), int(c)): float(r) for a, b, c, r in zip(gpu["segment"], gpu["template"], gpu["lag"], gpu["rho"])}
    o = {(int(a), int(b), int(c)): float(r) for a, b, c, r in zip(orc["segment"], orc["template"], orc["lag"], orc["rho"])}
    band = 0
    for key in o.keys() - g.keys():
        s, j, _ = key
        sg = sigma_o[s, j]
        assert abs(o[key]) <= kappa * sg + tol * sc[s, j], f"oracle tail {key} rho={o[key]} missing on the GPU"
        band += 1
    rows = {}
    for key in g.keys() - o.keys():
        s, j, n = key
        if (s, j) not in rows:
            rows[(s, j)] = oracle_rho(s, j)
        ro = rows[(s, j)][n]
        sg = sigma_o[s, j]
        assert abs(ro) >= kappa * sg - tol * sc[s, j], f"GPU tail {key} rho={g[key]} not a tail of the oracle ({ro})"
        band += 1
    common = g.keys() & o.keys()
    for key in common:
        s, j, _ = key
        assert abs(g[key] - o[key]) <= tol * sc[s, j], (key, g[key], o[key])
    return len(common), band


def max_rel_err(a, b, scale):
    """max |a - b| / scale over the last axis, as a float (scale broadcast per row; complex ok)."""
    return float(np.max(row_abs_err(a, b) / np.asarray(scale)))


def row_abs_err(a, b):
    """max |a - b| over the last axis, per row, in FP64 (complex ok)."""
    a, b = np.asarray(a), np.asarray(b)
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        d = np.abs(a.astype(np.complex128) - b.astype(np.complex128))
    else:
        d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    return np.max(d, axis=-1)


def strict_report(err_abs, sigma, floor):
    """Split per-correlation max errors by the relaxation cut.

    err_abs, sigma, floor: arrays of equal shape.  Returns a dict with the number of relaxed
    correlations, the worst err/sigma over the strict ones, the worst err/sigma and the worst
    err/(RELAX floor) over the relaxed ones."""
    err_abs, sigma, floor = (np.asarray(x, dtype=np.float64).ravel() for x in (err_abs, sigma, floor))
    rel = relaxed_mask(sigma, floor)
    out = {"n": int(err_abs.size), "n_relaxed": int(rel.sum()),
           "strict_max_err_over_sigma": float(np.max(err_abs[~rel] / sigma[~rel])) if (~rel).any() else 0.0}
    if rel.any():
        with np.errstate(divide="ignore"):
            out["relaxed_max_err_over_sigma"] = float(np.max(err_abs[rel] / sigma[rel]))
        out["relaxed_max_err_over_scale"] = float(np.max(err_abs[rel] / (RELAX * floor[rel])))
    return out


def sigma_floor(w, y):
    """Input scale of a correlation, ||w||_2 * rms(y): the sigma the template would have against
    white data of y's power.  Finite-precision FFT error is proportional to this scale, so a
    template whose sigma is tiny because it lies outside the data band (sigma << this scale)
    is held to tol * RELAX * this scale instead of tol * sigma."""
    w = np.asarray(w, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.sqrt(np.dot(w, w)) * np.sqrt(np.mean(y * y)))
