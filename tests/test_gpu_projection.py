"""Per-lag max projection (Sec. 3.3, Eqs. 13-17) on the GPU against the oracle's projection.

Several answers can be correct where two templates' significances agree within the
tolerance, so the test compares what is unique (the set of lags, the maximal
significance per lag) and checks that the GPU's winner is valid (its oracle significance
is within the tolerance of the maximum, with the same sign of rho)."""
import os

import numpy as np
import pytest

import oracle
from synthetic import get_workload, make_segment
from tests.parity import TOL, sigma_floor, tol_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bfs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_01609_amd import build as b

    if not os.path.exists(b.LIB):
        b.build()
    from paper_1708_01609_amd import bfsearch

    return bfsearch


def compare_projection(gpu, segs, temps, kappa, tol, out, floor=None):
    """gpu: PEAK_DTYPE records; out: oracle.search(...) result.  Returns (common, band_only).

    tol is in units of sigma; with floor ([S, K] sigma_floor values) a template far outside the
    data band has the tolerance tol * tol_scale(sigma, floor) / sigma in units of its sigma."""
    sig = out["sigma"]
    tsig = tol * tol_scale(sig, floor) / sig  # [S, K] tolerance of rho / sigma
    orc = oracle.max_projection(out["tails"], sig)
    by_key = {}
    for s, j, n, r in zip(out["tails"]["segment"], out["tails"]["template"], out["tails"]["lag"], out["tails"]["rho"]):
        by_key.setdefault((int(s), int(n)), {})[int(j)] = float(r) / sig[int(s), int(j)]
    rows = {}

    def snr_o(s, j, n):
        d = by_key.get((s, n), {})
        if j in d:
            return d[j]
        if (s, j) not in rows:
            rows[(s, j)] = oracle.correlate_fft(np.asarray(segs[s], np.float64), temps[j]) / sig[s, j]
        return float(rows[(s, j)][n])

    g = {(int(s), int(n)): (int(j), float(v)) for s, n, j, v in zip(gpu["segment"], gpu["lag"], gpu["template"], gpu["snr"])}
    o = {(int(s), int(n)): (int(j), float(v)) for s, n, j, v in zip(orc["segment"], orc["lag"], orc["template"], orc["snr"])}
    band = 0
    for key in o.keys() - g.keys():  # every oracle tail at this lag sits in the band
        s = key[0]
        assert all(abs(v) <= kappa + tsig[s, j] for j, v in by_key[key].items()), (key, by_key[key])
        band += 1
    for key in g.keys() - o.keys():  # the GPU's winner is a tail only within the band
        s, n = key
        assert abs(snr_o(s, g[key][0], n)) >= kappa - tsig[s, g[key][0]], (key, g[key])
        band += 1
    for key in g.keys() & o.keys():
        s, n = key
        jg, vg = g[key]
        jo, vo = o[key]
        t = max(tsig[s, jg], tsig[s, jo])
        assert abs(abs(vg) - abs(vo)) <= t + 2e-6 * abs(vo), (key, g[key], o[key])
        vj = snr_o(s, jg, n)
        assert abs(vj) >= abs(vo) - t - 2e-6 * abs(vo) and np.sign(vj) == np.sign(vg), (key, g[key], o[key], vj)
    return len(g.keys() & o.keys()), band


def _grid_run(bfs, w, segs, prec, **kw):
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    dt = np.float64 if prec == "f64" else np.float32
    lens = [len(y) for y in segs]
    flat = torch.from_numpy(np.concatenate(segs).astype(dt)).cuda()
    with bfs.Plan(max(lens), w.fs, kappa=w.kappa, grid=grid, precision=prec, project=True, n_min=min(lens),
                  **kw) as plan:
        with plan.filter(flat, lengths=lens) as job:
            peaks, total = job.fetch_projection()
            with pytest.raises(bfs.BfsError):
                job.fetch_tails()
    assert total == len(peaks)
    return peaks


def test_projection_c1_fp64(bfs):
    w = get_workload("C1")
    y, _ = make_segment(w, 0)
    peaks = _grid_run(bfs, w, [y], "f64")
    f0, fd, tau = w.template_params()
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    out = oracle.search([y], temps, w.kappa)
    common, band = compare_projection(peaks, [y], temps, w.kappa, TOL["f64"], out)
    orc = oracle.max_projection(out["tails"], out["sigma"])
    # FP64 on both sides: the same winners except where two agree to FP32 (the key's precision)
    same = np.sum(peaks["template"] == orc["template"]) if len(peaks) == len(orc) else 0
    print(f"C1 projection: {len(peaks)} lags, {common} common, {band} band-only, {same} identical winners")
    assert common > 50 and band <= 2 and same >= len(orc) - 2


def test_projection_c2_fp32(bfs):
    w = get_workload("C2")
    y, _ = make_segment(w, 0)
    peaks = _grid_run(bfs, w, [y], "f32")
    f0, fd, tau = w.template_params()
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    out = oracle.search([y.astype(np.float64)], temps, w.kappa)
    common, band = compare_projection(peaks, [y], temps, w.kappa, TOL["f32"], out)
    print(f"C2 projection: {len(peaks)} lags from {len(out['tails'])} oracle tails, {common} common, {band} band-only")
    assert common >= 0.99 * len(oracle.max_projection(out["tails"], out["sigma"]))
    assert len(peaks) < len(out["tails"])


def test_projection_uneven_graph_matches_eager_and_oracle(bfs):
    w0 = get_workload("C4")
    segs = [make_segment(w0, s)[0] for s in range(5)]

    class W:  # C4's shapes on a small grid
        n_f0, n_fdot, f0_range, fdot_range, taus, fs, kappa = 8, 8, w0.f0_range, w0.fdot_range, w0.taus, w0.fs, 4.5

    eager = _grid_run(bfs, W, segs, "f32")
    graph = _grid_run(bfs, W, segs, "f32", graph=True)
    assert np.array_equal(eager, graph)
    f0 = np.repeat(np.linspace(*W.f0_range, 8), 8)
    fd = np.tile(np.linspace(*W.fdot_range, 8), 8)
    tau = np.array([W.taus[j % 3] for j in range(64)])
    temps = oracle.template_bank(f0, fd, tau, W.fs)
    out = oracle.search([y.astype(np.float64) for y in segs], temps, W.kappa)
    # the grid's lowest chirps lie far outside the data band (sigma ~1e-3 of the input
    # scale): their tolerance scales with sigma_floor, as in the dense parity tests
    floor = np.array([[sigma_floor(t, y) for t in temps] for y in segs])
    common, band = compare_projection(eager, segs, temps, W.kappa, TOL["f32"], out, floor)
    print(f"uneven projection: {len(eager)} lags, {common} common, {band} band-only")
    assert common > 0 and band <= max(2, common // 100)
