"""Detector pairs on the GPU (Sec. 3.2 step (i); Sec. 5, Table 3).

Both channels of a pair go through one complex inverse transform (real part:
channel 2p, imaginary part: channel 2p + 1).  Every result is compared with the
oracle's single-channel correlations of the same seeded inputs; coincidences
with the oracle's coincidences of the same projections.
"""
import os

import numpy as np
import pytest

import oracle
from synthetic import bandlimited_noise, get_workload, make_segment, seeded_rng, unit_hann_chirp
from tests.parity import TOL, compare_tails, row_abs_err, sigma_floor, strict_report, tol_scale
from tests.test_gpu_projection import compare_projection

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


def _dev(y, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(np.atleast_2d(y).astype(dtype))).cuda()


SIZES = [("f32", 1 << p) for p in range(10, 17)] + [("f64", 1 << p) for p in range(10, 14)]


@pytest.mark.parametrize("prec,n", SIZES, ids=[f"{p}-N{n}" for p, n in SIZES])
def test_pair_dense_rho_and_sigma_match_oracle(bfs, prec, n):
    # 2 pairs of white noise with DC offsets of opposite sign (C_0 and C_{N/2} nonzero in both
    # channels) against templates of lengths 1, 7, N/4 and N
    rng = np.random.default_rng(n + (100 if prec == "f32" else 101))
    dtype = np.float64 if prec == "f64" else np.float32
    ys = np.stack([(rng.standard_normal(n) + (0.25 if s % 2 else -0.4)).astype(dtype) for s in range(4)])
    temps = [rng.standard_normal(l) for l in (1, 7, n // 4, n)]
    bank = np.zeros((len(temps), n))
    for j, w in enumerate(temps):
        bank[j, :len(w)] = w
    with bfs.Plan(n, 4096.0, kappa=5.0, templates=bank, precision=prec, pairs=True) as plan:
        rho_g, sig_g = plan.correlate_dense(_dev(ys, dtype))
        rho_g, sig_g = rho_g.cpu().numpy(), sig_g.cpu().numpy()
    bw = [b.astype(dtype).astype(np.float64) for b in bank]
    rho_o = np.stack([oracle.correlate_fft(y.astype(np.float64), np.array(bw)) for y in ys])
    sig_o = oracle.sigma_time(rho_o)
    err = float(np.max(row_abs_err(rho_g, rho_o) / sig_o))
    print(f"pairs {prec} N={n}: max |rho_gpu - rho_oracle| / sigma = {err:.3e}")
    assert err <= TOL[prec]
    assert np.max(np.abs(sig_g - sig_o) / sig_o) <= TOL[prec]


@pytest.mark.parametrize("n", [1 << 13, 1 << 14, 1 << 16], ids=lambda n: f"N{n}")
def test_every_pair_kernel_candidate_matches_oracle(bfs, n):
    rng = np.random.default_rng(n + 17)
    ys = np.stack([(rng.standard_normal(n) + 0.25).astype(np.float32) for _ in range(2)])
    temps = [rng.standard_normal(l) for l in (1, 33, n // 4, n)]
    bank = np.zeros((len(temps), n))
    for j, w in enumerate(temps):
        bank[j, :len(w)] = w
    bw = np.array([b.astype(np.float32).astype(np.float64) for b in bank])
    rho_o = np.stack([oracle.correlate_fft(y.astype(np.float64), bw) for y in ys])
    sig_o = oracle.sigma_time(rho_o)
    with bfs.Plan(n, 4096.0, kappa=5.0, templates=bank, precision="f32", pairs=True) as plan:
        count = plan.kernel_info()["n_candidates"]
    for c in range(1, count + 1):
        with bfs.Plan(n, 4096.0, kappa=5.0, templates=bank, precision="f32", candidate=c, pairs=True) as plan:
            rho_g, sig_g = plan.correlate_dense(_dev(ys))
            rho_g, sig_g = rho_g.cpu().numpy(), sig_g.cpu().numpy()
        err = float(np.max(row_abs_err(rho_g, rho_o) / sig_o))
        print(f"pairs N={n} candidate {c}: max err / sigma = {err:.3e}")
        assert err <= TOL["f32"] and np.max(np.abs(sig_g - sig_o) / sig_o) <= TOL["f32"]


def _c2_pairs(count):
    """count pairs of C2-shaped segments: channel 0 and channel 1 of segment indices 0..count-1."""
    w = get_workload("C2")
    a = [make_segment(w, s, channel=0)[0] for s in range(count)]
    b = [make_segment(w, s, channel=1)[0] for s in range(count)]
    return w, oracle.pair_segments(a, b)


def test_pair_tails_and_sigma_match_oracle_and_single_plan(bfs):
    # 2 pairs at N = 2^16 against 1024 chirps of the C2 ranges, kappa = 5: the pair plan's tails
    # and sigma against the oracle, and the same tails as the single-segment plan outside the band
    w, segs = _c2_pairs(2)
    grid = bfs.Grid(64, 16, w.f0_range, w.fdot_range, w.taus)
    f0, fd, tau = oracle.grid_params(64, 16, w.f0_range, w.fdot_range, w.taus)
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    ys = _dev(np.stack(segs))
    res = {}
    for pairs in (True, False):
        with bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision="f32", pairs=pairs) as plan:
            with plan.filter(ys) as job:
                res[pairs] = (job.fetch_tails()[0], job.fetch_sigma())
    tails, sig = res[True]
    out = oracle.search(segs, temps, w.kappa)
    floor = np.array([[sigma_floor(t, y) for t in temps] for y in segs])
    assert np.max(np.abs(sig - out["sigma"]) / tol_scale(out["sigma"], floor)) <= TOL["f32"]
    common, band = compare_tails(tails, out["tails"], out["sigma"], w.kappa, TOL["f32"],
                                 lambda s, j: oracle.correlate_fft(segs[s].astype(np.float64), temps[j]), floor)
    assert common >= 0.99 * len(out["tails"]) and len(out["tails"]) > 50
    # the single-segment plan, same inputs: sigma within the tolerance, tails equal outside the band
    compare_tails(res[False][0], tails, res[True][1], w.kappa, 2 * TOL["f32"],
                  lambda s, j: oracle.correlate_fft(segs[s].astype(np.float64), temps[j]), floor)
    print(f"pairs: {len(tails)} tails, common with oracle {common}, band-only {band}")


def test_pair_dense_c2_bank_strict(bfs):
    # one C2 pair against the whole 8192-chirp bank, every rho: strict 1e-4 sigma except the
    # templates far outside the data band
    w, segs = _c2_pairs(1)
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    f0, fd, tau = w.template_params()
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    ys = _dev(np.stack(segs))
    errs, sigs, floors = [], [], []
    with bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision="f32", pairs=True) as plan:
        for j0 in range(0, w.n_templates, 512):
            rho_g, _ = plan.correlate_dense(ys, first=j0, count=512)
            rho_g = rho_g.cpu().numpy()
            for s in range(2):
                ro = oracle.correlate_fft(segs[s].astype(np.float64), np.array(temps[j0:j0 + 512]))
                errs.append(row_abs_err(rho_g[s], ro))
                sigs.append(oracle.sigma_time(ro))
                floors.append([sigma_floor(t, segs[s]) for t in temps[j0:j0 + 512]])
            del rho_g
    rep = strict_report(np.concatenate(errs), np.concatenate(sigs), np.concatenate(floors))
    print(f"pairs dense C2 bank, both channels: {rep}")
    assert rep["strict_max_err_over_sigma"] <= TOL["f32"]
    assert np.all(np.concatenate(errs) <= TOL["f32"] * tol_scale(np.concatenate(sigs), np.concatenate(floors)))


def test_pair_uneven_lengths_graph_replays_and_tiles(bfs):
    # pairs of 2^14, 2^15 and 2^16 samples in one call (each pair's channels of equal length):
    # every tile order and every graph replay gives the eager tile-1 result bitwise, and that
    # matches the oracle
    w = get_workload("C4")
    lens = [1 << 15, 1 << 14, 1 << 16, 1 << 14, 1 << 15]
    segs = []
    for p, n in enumerate(lens):
        segs += [bandlimited_noise(n, w.fs, seeded_rng(40, c, p, "noise")).astype(np.float32) for c in (0, 1)]
    seg_lens = [len(y) for y in segs]
    grid = bfs.Grid(8, 8, w.f0_range, w.fdot_range, w.taus)
    f0, fd, tau = oracle.grid_params(8, 8, w.f0_range, w.fdot_range, w.taus)
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    flat = torch.from_numpy(np.concatenate(segs)).cuda()
    res = {}
    for tile in (1, 2, 3, 8):
        with bfs.Plan(1 << 16, w.fs, kappa=4.5, grid=grid, precision="f32", n_min=1 << 14, pairs=True,
                      tile=tile) as plan:
            with plan.filter(flat, lengths=seg_lens) as job:
                res[tile] = (job.fetch_tails()[0], job.fetch_sigma())
    for tile, (t, sg) in res.items():
        assert np.array_equal(t, res[1][0]) and np.array_equal(sg, res[1][1]), tile
    with bfs.Plan(1 << 16, w.fs, kappa=4.5, grid=grid, precision="f32", n_min=1 << 14, pairs=True,
                  graph=True) as plan:
        for rep in range(3):
            _ = torch.randn(1 << 18, device="cuda").sum().item()
            with plan.filter(flat, lengths=seg_lens) as job:
                t, sg = job.fetch_tails()[0], job.fetch_sigma()
            assert np.array_equal(t, res[1][0]) and np.array_equal(sg, res[1][1]), rep
    out = oracle.search(segs, temps, 4.5)
    floor = np.array([[sigma_floor(tm, y) for tm in temps] for y in segs])
    assert np.max(np.abs(res[1][1] - out["sigma"]) / tol_scale(out["sigma"], floor)) <= TOL["f32"]
    common, band = compare_tails(res[1][0], out["tails"], out["sigma"], 4.5, TOL["f32"],
                                 lambda s, j: oracle.correlate_fft(segs[s].astype(np.float64), temps[j]), floor)
    assert common > 100


def test_pair_projection_and_coincidences(bfs):
    # two pairs at N = 2^16; pair 0 carries the same chirp (SNR 14) in both channels at one
    # offset.  The projection of every channel matches the oracle's; the coincidences are
    # exactly the oracle's coincidences of the GPU's own projection (the window is decided in
    # FP64 on both sides) and agree with the oracle's projection outside near-ties
    w = get_workload("C2")
    fs, n, off, L = w.fs, w.n, 20000, 4096
    chirp = 14.0 * unit_hann_chirp(900.0, 120.0, L, fs)
    segs = []
    for p in range(2):
        for c in range(2):
            y = bandlimited_noise(n, fs, seeded_rng(41, c, p, "noise"))
            if p == 0:
                y[off:off + L] += chirp
            segs.append(y.astype(np.float32))
    nf0, nfd = 64, 32
    grid = bfs.Grid(nf0, nfd, w.f0_range, w.fdot_range, w.taus)
    f0, fd, tau = oracle.grid_params(nf0, nfd, w.f0_range, w.fdot_range, w.taus)
    temps = oracle.template_bank(f0, fd, tau, fs)
    delta = 50.0
    with bfs.Plan(n, fs, kappa=4.0, grid=grid, precision="f32", pairs=True, project=True,
                  coinc_delta_hz=delta) as plan:
        with plan.filter(_dev(np.stack(segs))) as job:
            peaks, npk = job.fetch_projection()
            coinc, nco = job.fetch_coincidences()
    assert npk == len(peaks) and nco == len(coinc)
    out = oracle.search(segs, temps, 4.0)
    floor = np.array([[sigma_floor(t, y) for t in temps] for y in segs])
    common, band = compare_projection(peaks, segs, temps, 4.0, TOL["f32"], out, floor)
    gp = np.zeros(len(peaks), dtype=oracle.PEAK_DTYPE)
    for f in ("segment", "lag", "template"):
        gp[f] = peaks[f]
    gp["snr"] = peaks["snr"].astype(np.float64)
    want = oracle.coincidences(gp, f0, delta)
    assert len(coinc) == len(want) > 0
    for f in ("pair", "lag", "template_a", "template_b"):
        assert np.array_equal(coinc[f], want[f]), f
    assert np.array_equal(coinc["snr_a"], want["snr_a"].astype(np.float32))
    assert np.array_equal(coinc["snr_b"], want["snr_b"].astype(np.float32))
    # against the oracle's own projection: the same coincidences wherever both projections agree
    orc = oracle.coincidences(oracle.max_projection(out["tails"], out["sigma"]), f0, delta)
    g = {(int(p), int(n)) for p, n in zip(coinc["pair"], coinc["lag"])}
    o = {(int(p), int(n)) for p, n in zip(orc["pair"], orc["lag"])}
    gw = {(int(s), int(n)): int(j) for s, n, j in zip(peaks["segment"], peaks["lag"], peaks["template"])}
    op = oracle.max_projection(out["tails"], out["sigma"])
    ow = {(int(s), int(n)): int(j) for s, n, j in zip(op["segment"], op["lag"], op["template"])}
    for p, n in g ^ o:  # a differing coincidence needs a differing winner (a near-tie) in a channel
        assert any(gw.get((2 * p + c, n)) != ow.get((2 * p + c, n)) for c in (0, 1)), (p, n)
    near = [c for c in coinc if c["pair"] == 0 and abs(int(c["lag"]) - off) <= 64]
    print(f"pairs projection: {npk} lags, common {common}, band-only {band}; coincidences {nco} "
          f"(oracle's own projection {len(orc)}, {len(g ^ o)} differ at near-ties), {len(near)} at the chirp")
    assert len(near) > 0 and len(g & o) >= 0.9 * len(o)


def test_pair_plans_reject_unpaired_segments(bfs):
    with bfs.Plan(4096, 4096.0, kappa=4.0, templates=np.ones((2, 64)), precision="f32", pairs=True,
                  n_min=2048) as plan:
        y = torch.zeros(1 << 15, device="cuda")
        for lens in ([4096], [4096, 4096, 4096], [4096, 2048], [2048, 2048, 4096, 2048]):
            with pytest.raises(bfs.BfsError) as e:
                plan.filter(y, lengths=lens)
            assert e.value.status == bfs.BFS_ERR_INVALID_ARG, lens
        with plan.filter(y, lengths=[2048, 2048, 4096, 4096]) as job:  # well-formed pairs
            assert job.fetch_sigma().shape == (4, 2)
        with pytest.raises(bfs.BfsError):  # no coincidence window on this plan
            with plan.filter(y, lengths=[2048, 2048]) as job:
                job.fetch_coincidences()
