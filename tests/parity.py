"""Helpers for GPU-vs-oracle parity checks (tolerances in units of the oracle's sigma)."""
from __future__ import annotations

import numpy as np

# Tolerances on |rho_gpu - rho_oracle| / sigma_oracle and on the tail band:
#   FP64 path 1e-9, FP32 path 1e-4, FP16-stored spectra 2e-3.
TOL = {"f64": 1e-9, "f32": 1e-4, "f32-w16f": 2e-3, "f32-w16b": 2e-2}


def compare_tails(gpu, orc, sigma_o, kappa, tol, oracle_rho, floor=None):
    """Tail sets must agree outside a +-tol*sigma band around kappa*sigma.

    gpu: records with segment/template/lag/rho; orc: oracle TAIL_DTYPE records;
    sigma_o: [S, K] oracle sigma; oracle_rho(s, j) -> oracle rho row (for GPU
    tails the oracle did not report); floor: optional [S, K] sigma_floor values
    (the band and value tolerance use max(sigma, floor)).  Returns
    (n_common, n_band_only).
    """
    sc = sigma_o if floor is None else np.maximum(sigma_o, floor)
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
    a, b = np.asarray(a), np.asarray(b)
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        d = np.abs(a.astype(np.complex128) - b.astype(np.complex128))
    else:
        d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    return float(np.max(d / np.asarray(scale)[..., None]))


def sigma_floor(w, y):
    """Input scale of a correlation, ||w||_2 * rms(y): the sigma the template would have against
    white data of y's power.  Finite-precision FFT error is proportional to this scale, so a
    template whose sigma is tiny because it lies outside the data band (sigma << this scale)
    is held to tol * this scale instead of tol * sigma."""
    w = np.asarray(w, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.sqrt(np.dot(w, w)) * np.sqrt(np.mean(y * y)))
