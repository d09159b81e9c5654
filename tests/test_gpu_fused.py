"""GPU parity of fused synthesis (templates made per correlation, no resident bank).

The fused kernel synthesises each chirp on chip, transforms it and correlates
it; it must meet the FP32 bar against the FP64 oracle like the resident path:
|rho error| <= 1e-4 sigma for every correlation whose sigma is at least
0.1 sigma_floor, 1e-5 sigma_floor below (tests/parity.py), tail sets equal
outside the tolerance band.  Expected values come only from oracle/.
"""
import os

import numpy as np
import pytest

import oracle
from synthetic import get_workload, make_segment
from tests.parity import TOL, compare_tails, relaxed_mask, row_abs_err, sigma_floor, strict_report, tol_scale
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


def _dev(y):
    return torch.from_numpy(np.ascontiguousarray(np.atleast_2d(y).astype(np.float32))).cuda()


def _check_dense(plan, y, temps, first=0, block=1024):
    """Dense rho and sigma of templates first.. of the plan against the oracle; returns the
    strict report and the per-template errors."""
    y64 = np.asarray(y, np.float64)
    k = len(temps)
    err, sg, so = np.empty(k), np.empty(k), np.empty(k)
    for j0 in range(0, k, block):
        c = min(block, k - j0)
        rho_g, sig_g = plan.correlate_dense(_dev(y), first=first + j0, count=c)
        rho_g, sig_g = rho_g.cpu().numpy()[0], sig_g.cpu().numpy()[0]
        rho_o = oracle.correlate_fft(y64, np.array(temps[j0:j0 + c]))
        err[j0:j0 + c] = row_abs_err(rho_g, rho_o)
        sg[j0:j0 + c] = sig_g
        so[j0:j0 + c] = oracle.sigma_time(rho_o)
    floor = np.array([sigma_floor(t, y) for t in temps])
    rep = strict_report(err, so, floor)
    assert rep["strict_max_err_over_sigma"] <= TOL["f32"], rep
    assert np.all(err <= TOL["f32"] * tol_scale(so, floor))
    assert np.all(np.abs(sg - so) <= TOL["f32"] * tol_scale(so, floor))
    return rep


# lengths with a fused kernel; per length one duration whose first pass is pruned (template
# within two rows of the transform's first pass) and one that needs every row
FUSED = [(1 << 10, 0.03), (1 << 10, 0.25), (1 << 13, 0.25), (1 << 13, 1.0), (1 << 16, 1.0), (1 << 16, 8.0)]


@pytest.mark.parametrize("n,tau", FUSED, ids=[f"N{n}-tau{t}" for n, t in FUSED])
def test_fused_dense_matches_oracle(bfs, n, tau):
    rng = np.random.default_rng(n + int(100 * tau))
    y = (rng.standard_normal(n) + 0.25).astype(np.float32)  # DC offset: C_0, C_{N/2} nonzero
    grid = bfs.Grid(6, 5, (350.0, 1900.0), (-300.0, 300.0), (tau,))
    with bfs.Plan(n, 4096.0, kappa=5.0, grid=grid, precision="f32", fused=True) as plan:
        info = plan.kernel_info()
        assert info["fused"] and plan.bank_bytes == 0
        f0, fd, taus = oracle.grid_params(6, 5, (350.0, 1900.0), (-300.0, 300.0), (tau,))
        temps = oracle.template_bank(f0, fd, taus, 4096.0)
        rep = _check_dense(plan, y, temps)
    print(f"fused N={n} tau={tau}: rows {info['fused_rows']}, {rep}")


def test_fused_c2_matches_oracle(bfs):
    # C2 at full size: every rho of all 8192 templates, and the tail set of the filter path
    w = get_workload("C2")
    y, _ = make_segment(w, 0)
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    f0, fd, tau = w.template_params()
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    out = oracle.search([y.astype(np.float64)], temps, w.kappa)
    floor = np.array([[sigma_floor(t, y) for t in temps]])
    with bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision="f32", fused=True) as plan:
        with plan.filter(_dev(y)) as job:
            tails, total = job.fetch_tails()
            sig = job.fetch_sigma()
        rep = _check_dense(plan, y, temps)
    assert total == len(tails) and total > 100
    assert np.all(np.abs(sig - out["sigma"]) <= TOL["f32"] * tol_scale(out["sigma"], floor))
    common, band = compare_tails(tails, out["tails"], out["sigma"], w.kappa, TOL["f32"],
                                 lambda s, j: oracle.correlate_fft(y.astype(np.float64), temps[j]), floor)
    print(f"fused C2: dense {rep}; tails {total}, common {common}, band-only {band}")
    assert common >= 0.99 * len(out["tails"])


def test_fused_c3_subset_matches_oracle(bfs):
    # C3's bank of 2^20 chirps without residency: templates 0..4095 against the oracle
    w = get_workload("C3")
    y, _ = make_segment(w, 0)
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    f0, fd, tau = w.template_params()
    temps = oracle.template_bank(f0, fd, tau, w.fs, ids=range(4096))
    with bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision="f32", fused=True) as plan:
        assert plan.bank_bytes == 0
        rep = _check_dense(plan, y, temps)
    print(f"fused C3 templates 0..4095: {rep}")


def test_bank_over_budget_falls_back_to_fused_synthesis(bfs):
    # a resident FP32 C2 bank takes 2 GiB; with a 1 GiB budget the plan synthesises per correlation
    w = get_workload("C2")
    y, _ = make_segment(w, 0)
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    with bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision="f32", hbm_budget_bytes=1 << 30) as plan:
        assert plan.kernel_info()["fused"] and plan.bank_bytes == 0
        with plan.filter(_dev(y)) as job:
            tails, total = job.fetch_tails()
    with bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision="f32") as plan:
        assert not plan.kernel_info()["fused"]
        with plan.filter(_dev(y)) as job:
            ref, ref_total = job.fetch_tails()
    # fused and resident round differently: their tail sets agree outside the tolerance band
    f0, fd, tau = w.template_params()
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    out = oracle.search([y.astype(np.float64)], temps, w.kappa)
    floor = np.array([[sigma_floor(t, y) for t in temps]])
    for t in (tails, ref):
        compare_tails(t, out["tails"], out["sigma"], w.kappa, TOL["f32"],
                      lambda s, j: oracle.correlate_fft(y.astype(np.float64), temps[j]), floor)
    assert abs(total - ref_total) <= 2


def test_fused_symmetric_projection_and_band(bfs):
    # the plan options ride on the fused kernel too: time-symmetric chirps (dense vs oracle),
    # the per-lag max projection and a finite tail band (vs the oracle's)
    n, fs = 1 << 13, 4096.0
    w = get_workload("C1")
    y, _ = make_segment(w, 0)
    y = y.astype(np.float32)
    args = (8, 8, (400.0, 1800.0), (-200.0, 200.0), (0.25,))
    f0, fd, tau = oracle.grid_params(*args)
    sym = bfs.Grid(*args, symmetric=True)
    with bfs.Plan(n, fs, kappa=4.0, grid=sym, precision="f32", fused=True) as plan:
        _check_dense(plan, y, oracle.template_bank(f0, fd, tau, fs, symmetric=True))
    temps = oracle.template_bank(f0, fd, tau, fs)
    out = oracle.search([y.astype(np.float64)], temps, 4.0)
    with bfs.Plan(n, fs, kappa=4.0, grid=bfs.Grid(*args), precision="f32", fused=True, project=True) as plan:
        with plan.filter(_dev(y)) as job:
            peaks, _ = job.fetch_projection()
    common, band = compare_projection(peaks, [y], temps, 4.0, TOL["f32"], out)
    assert common > 50 and band <= 2
    band_out = oracle.search([y.astype(np.float64)], temps, 3.0, kappa_hi=3.5)
    with bfs.Plan(n, fs, kappa=3.0, kappa_hi=3.5, grid=bfs.Grid(*args), precision="f32", fused=True,
                  tail_capacity=1 << 18) as plan:
        with plan.filter(_dev(y)) as job:
            tails, total = job.fetch_tails()
    g = set(zip(tails["template"].tolist(), tails["lag"].tolist()))
    o = set(zip(band_out["tails"]["template"].tolist(), band_out["tails"]["lag"].tolist()))
    print(f"fused band: {total} tails, oracle {len(o)}, differing {len(g ^ o)}")
    assert total > 1000 and len(g ^ o) <= max(4, len(o) // 1000)
