"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every comparison is element by element on the same seeded inputs; tolerances
are in units of the oracle's sigma (tests/parity.py).  Inputs come from the
synthetic generators or seeded numpy draws; expected values only from oracle/.
"""
import os

import numpy as np
import pytest

import oracle
from synthetic import get_workload, make_segment
from tests.parity import (BF16_MODEL_BOUND, TOL, compare_tails, max_rel_err, relaxed_mask, row_abs_err,
                          sigma_floor, strict_report, tol_scale)

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


def _dev(y, dtype):
    return torch.from_numpy(np.ascontiguousarray(np.atleast_2d(y).astype(dtype))).cuda()


def _oracle_dense(ys, temps):
    """[S][K][N] oracle rho and [S][K] sigma for explicit templates."""
    rho = np.stack([oracle.correlate_fft(np.asarray(y, np.float64), np.array(
        [np.pad(w, (0, len(y) - len(w))) for w in temps])) for y in ys])
    return rho, oracle.sigma_time(rho)


SIZES = [("f32", 1 << p) for p in range(10, 18)] + [("f64", 1 << p) for p in range(10, 15)]


@pytest.mark.parametrize("prec,n", SIZES, ids=[f"{p}-N{n}" for p, n in SIZES])
def test_dense_rho_and_sigma_match_oracle(bfs, prec, n):
    # white noise with a DC offset (so C_0 and C_{N/2} are nonzero) against templates of
    # lengths 1, 7, N/4 and N; ragged K = 4 correlations per segment, 2 segments
    rng = np.random.default_rng(n + (0 if prec == "f32" else 1))
    dtype = np.float64 if prec == "f64" else np.float32
    ys = [(rng.standard_normal(n) + 0.25).astype(dtype) for _ in range(2)]
    temps = [rng.standard_normal(l) for l in (1, 7, n // 4, n)]
    lmax = max(len(w) for w in temps)
    bank = np.zeros((len(temps), lmax))
    for j, w in enumerate(temps):
        bank[j, :len(w)] = w
    with bfs.Plan(n, 4096.0, kappa=5.0, templates=bank, precision=prec) as plan:
        rho_g, sig_g = plan.correlate_dense(_dev(np.stack(ys), dtype))
        torch.cuda.synchronize()
        rho_g, sig_g = rho_g.cpu().numpy(), sig_g.cpu().numpy()
    rho_o, sig_o = _oracle_dense([y.astype(np.float64) for y in ys],
                                 [b.astype(dtype).astype(np.float64) for b in bank])
    tol = TOL[prec]
    err = max_rel_err(rho_g.reshape(-1, n), rho_o.reshape(-1, n), sig_o.reshape(-1))
    print(f"{prec} N={n}: max |rho_gpu - rho_oracle| / sigma = {err:.3e}")
    assert err <= tol, f"max |rho_gpu - rho_oracle| / sigma = {err:.3e}"
    assert np.max(np.abs(sig_g - sig_o) / sig_o) <= tol


@pytest.mark.parametrize("n", [1 << 16, 1 << 17])
def test_impulse_closed_form_on_gpu(bfs, n):
    # y = delta at n0 => rho[n] = w[(n0 - n) mod N] (FP32)
    n0 = 12345
    w = np.random.default_rng(3).standard_normal(4096)
    y = np.zeros(n, np.float32)
    y[n0] = 1.0
    with bfs.Plan(n, 4096.0, kappa=5.0, templates=w[None, :], precision="f32") as plan:
        rho, sig = plan.correlate_dense(_dev(y, np.float32))
        rho = rho.cpu().numpy()[0, 0]
    wpad = np.zeros(n)
    wpad[:len(w)] = w.astype(np.float32)
    expect = wpad[(n0 - np.arange(n)) % n]
    sigma = np.sqrt(np.mean(expect ** 2))
    assert np.max(np.abs(rho - expect)) <= 1e-4 * sigma


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_grid_template_spectra_match_oracle(bfs, prec):
    # a2 + a3: chirps synthesised and transformed on the device vs the oracle's closed form + rfft
    w = get_workload("C1")
    n = w.n
    f0, fd, tau = w.template_params()
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    with bfs.Plan(n, w.fs, kappa=w.kappa, grid=grid, precision=prec) as plan:
        spec = plan.spectra().cpu().numpy()
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    ref = np.fft.rfft(np.array([np.pad(t, (0, n - len(t))) for t in temps]), axis=-1)
    scale = np.max(np.abs(ref), axis=-1)
    err = max_rel_err(spec, ref, scale)
    print(f"{prec}: max |W_gpu - W_oracle| / max|W| = {err:.3e}")
    assert err <= (1e-12 if prec == "f64" else 2e-6), err


@pytest.mark.parametrize("name", ["C2", "C4"])
def test_segment_spectrum_matches_rfft(bfs, name):
    # C2 segment 0: N = 2^16; C4 segment 3: N = 2^17 (the split transform)
    w = get_workload(name)
    y, _ = make_segment(w, 3 if name == "C4" else 0)
    n = len(y)
    with bfs.Plan(n, w.fs, kappa=w.kappa, templates=np.ones((1, 16)), precision="f32") as plan:
        job = plan.filter(_dev(y, np.float32))
        spec = job.spectra().cpu().numpy()[0]
        job.release()
    ref = np.fft.rfft(y.astype(np.float64))
    assert np.max(np.abs(spec - ref)) <= 2e-6 * np.max(np.abs(ref))


def test_template_spectra_at_every_plan_length(bfs):
    # one plan over 2^14..2^17: the bank at each length is the rfft of the template zero-padded
    # to that length (durations 0.5, 1 and 2 s as in the batched workload)
    w = get_workload("C4")
    grid = bfs.Grid(4, 4, w.f0_range, w.fdot_range, w.taus)
    f0 = np.repeat(np.linspace(*w.f0_range, 4), 4)
    fd = np.tile(np.linspace(*w.fdot_range, 4), 4)
    tau = np.array([w.taus[j % len(w.taus)] for j in range(16)])
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    with bfs.Plan(1 << 17, w.fs, kappa=5.0, grid=grid, precision="f32", n_min=1 << 14) as plan:
        assert plan.n_min == 1 << 14
        for n in (1 << 14, 1 << 15, 1 << 16, 1 << 17):
            spec = plan.spectra(n=n).cpu().numpy()
            ref = np.fft.rfft(np.array([np.pad(t, (0, n - len(t))) for t in temps]), axis=-1)
            err = max_rel_err(spec, ref, np.max(np.abs(ref), axis=-1))
            assert err <= 2e-6, (n, err)


def _workload_run(bfs, name, n_templates=None):
    w = get_workload(name)
    y, inj = make_segment(w, 0)
    prec = w.dtype
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    plan = bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision=prec)
    job = plan.filter(_dev(y, np.float64 if prec == "f64" else np.float32))
    tails, total = job.fetch_tails()
    sig = job.fetch_sigma()
    job.release()
    return w, y, inj, plan, tails, total, sig


def test_c1_fp64_tails_and_sigma(bfs):
    # C1: N = 2^13, 64 chirps, SNR-20 injection, kappa = 4, FP64 on both sides
    w, y, inj, plan, tails, total, sig = _workload_run(bfs, "C1")
    f0, fd, tau = w.template_params()
    bank = oracle.template_bank(f0, fd, tau, w.fs)
    out = oracle.search([y], bank, w.kappa, keep_rho=True)
    assert total == len(tails)
    assert np.max(np.abs(sig - out["sigma"]) / out["sigma"]) <= TOL["f64"]
    common, band = compare_tails(tails, out["tails"], out["sigma"], w.kappa, TOL["f64"],
                                 lambda s, j: out["rho"][s][j])
    assert common > 50 and band <= 2
    plan.close()


@pytest.fixture(scope="module")
def c2_oracle():
    w = get_workload("C2")
    y, inj = make_segment(w, 0)
    f0, fd, tau = w.template_params()
    bank = oracle.template_bank(f0, fd, tau, w.fs)
    return w, y, bank, oracle.search([y], bank, w.kappa)


def _dense_blocks(plan, y_dev, y64, temps, first=0, block=1024):
    """Per template of temps (ids first.. of the plan): max |rho_gpu - rho_oracle| over every
    lag, sigma_gpu and the oracle's sigma, taken block by block through the dense diagnostic."""
    k = len(temps)
    err, sg, so = np.empty(k), np.empty(k), np.empty(k)
    for j0 in range(0, k, block):
        c = min(block, k - j0)
        rho_g, sig_g = plan.correlate_dense(y_dev, first=first + j0, count=c)
        rho_g, sig_g = rho_g.cpu().numpy()[0], sig_g.cpu().numpy()[0]
        rho_o = oracle.correlate_fft(y64, np.array(temps[j0:j0 + c]))
        err[j0:j0 + c] = row_abs_err(rho_g, rho_o)
        sg[j0:j0 + c] = sig_g
        so[j0:j0 + c] = oracle.sigma_time(rho_o)
        del rho_g, rho_o
    return err, sg, so


def test_c2_fp32_tails_sigma_and_dense_rho(bfs, c2_oracle):
    # C2 at full size in the launch configuration the bench times: N = 2^16, 8192 chirps,
    # kappa = 5.  Every rho of every template against the oracle: strict 1e-4 sigma wherever
    # sigma >= 0.1 sigma_floor, 1e-4 * 0.1 sigma_floor below (templates almost wholly outside
    # the data band, 138 of 8192 here)
    w, y, bank, out = c2_oracle
    w2, y2, inj, plan, tails, total, sig = _workload_run(bfs, "C2")
    assert np.array_equal(y, y2)
    assert total == len(tails) and total > 100

    def rho_row(s, j):
        return oracle.correlate_fft(y.astype(np.float64), bank[j])

    floor = np.array([[sigma_floor(bank[j], y) for j in range(w.n_templates)]])
    assert np.max(np.abs(sig - out["sigma"]) / tol_scale(out["sigma"], floor)) <= TOL["f32"]
    common, band = compare_tails(tails, out["tails"], out["sigma"], w.kappa, TOL["f32"], rho_row, floor)
    assert common >= 0.99 * len(out["tails"])
    err, sg, so = _dense_blocks(plan, _dev(y, np.float32), y.astype(np.float64), bank)
    rep = strict_report(err, so, floor[0])
    print(f"C2 dense rho, {w.n_templates} templates: {rep}; sigma max rel err (strict set) "
          f"{np.max(np.abs(sg - so)[~relaxed_mask(so, floor[0])] / so[~relaxed_mask(so, floor[0])]):.3e}; "
          f"common tails {common}, band-only {band}")
    assert rep["n_relaxed"] <= 200
    assert rep["strict_max_err_over_sigma"] <= TOL["f32"]
    assert np.all(err <= TOL["f32"] * tol_scale(so, floor[0]))
    assert np.all(np.abs(sg - so) <= TOL["f32"] * tol_scale(so, floor[0]))
    plan.close()


@pytest.mark.parametrize("prec", ["f32-w16f", "f32-w16b"], ids=["fp16-meets-2e-3", "bf16-misses-2e-3-within-error-model"])
def test_reduced_precision_spectra_error(bfs, prec):
    # precision form: template spectra stored 16-bit, FFT and accumulation FP32, sigma FP64; every
    # rho of all 8192 C2 templates against the oracle.  FP16 meets the 2e-3 sigma bar.  BF16's
    # 8-bit mantissa misses it (predicted ~1e-2 sigma worst case): held to the error model's bound
    # and reported, not passed under a widened bar.
    w = get_workload("C2")
    y, _ = make_segment(w, 0)
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    f0, fd, tau = w.template_params()
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    floor = np.array([sigma_floor(t, y) for t in temps])
    with bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision=prec) as plan:
        err, sg, so = _dense_blocks(plan, _dev(y, np.float32), y.astype(np.float64), temps)
    rep = strict_report(err, so, floor)
    sig_err = float(np.max(np.abs(sg - so) / tol_scale(so, floor)))
    meets = rep["strict_max_err_over_sigma"] <= TOL[prec] and np.all(err <= TOL[prec] * tol_scale(so, floor))
    print(f"{prec}: dense rho over 8192 templates {rep}; sigma err/scale {sig_err:.3e}; "
          f"meets 2e-3 sigma: {bool(meets)}")
    assert sig_err <= TOL[prec]
    if prec == "f32-w16f":
        assert meets
    else:
        assert rep["strict_max_err_over_sigma"] <= BF16_MODEL_BOUND
        assert np.all(err <= BF16_MODEL_BOUND * tol_scale(so, floor))


def test_kappa_zero_returns_every_lag(bfs):
    # kappa = 0: every nonzero lag is a tail, so the compacted list is the whole rho
    n = 1024
    rng = np.random.default_rng(9)
    y = rng.standard_normal(n).astype(np.float32)
    temps = rng.standard_normal((3, 100))
    with bfs.Plan(n, 4096.0, kappa=0.0, templates=temps, precision="f32", tail_capacity=4 * n) as plan:
        with plan.filter(_dev(y, np.float32)) as job:
            tails, total = job.fetch_tails()
    rho_o, sig_o = _oracle_dense([y.astype(np.float64)], [t.astype(np.float32).astype(np.float64) for t in temps])
    assert total == 3 * n
    assert np.array_equal(tails["template"], np.repeat(np.arange(3), n))
    assert np.array_equal(tails["lag"], np.tile(np.arange(n), 3))
    assert np.max(np.abs(tails["rho"] - rho_o[0].reshape(-1)) / np.repeat(sig_o[0], n)) <= TOL["f32"]


def test_tail_overflow_keeps_exact_total(bfs):
    n = 1024
    rng = np.random.default_rng(10)
    y = rng.standard_normal(n).astype(np.float32)
    temps = rng.standard_normal((4, 64))
    with bfs.Plan(n, 4096.0, kappa=1.0, templates=temps, precision="f32", tail_capacity=4 * n) as plan:
        with plan.filter(_dev(y, np.float32)) as job:
            full, total = job.fetch_tails()
            part, total2 = job.fetch_tails(capacity=10, allow_overflow=True)
            with pytest.raises(bfs.BfsError) as e:
                job.fetch_tails(capacity=10)
            assert e.value.status == bfs.BFS_ERR_TAIL_OVERFLOW
    assert total == len(full) == total2 > 10 and len(part) == 10
    # a device buffer smaller than the tail count: exact total, overflow reported
    with bfs.Plan(n, 4096.0, kappa=1.0, templates=temps, precision="f32", tail_capacity=7) as plan:
        with plan.filter(_dev(y, np.float32)) as job:
            part, total3 = job.fetch_tails(allow_overflow=True)
    assert total3 == total and len(part) == 7


def test_zero_segment_gives_zero_sigma_and_no_tails(bfs):
    n = 4096
    with bfs.Plan(n, 4096.0, kappa=3.0, templates=np.ones((2, 50)), precision="f32") as plan:
        with plan.filter(_dev(np.zeros(n), np.float32)) as job:
            tails, total = job.fetch_tails()
            sig = job.fetch_sigma()
    assert total == 0 and np.all(sig == 0.0)


def test_multi_segment_batch_equals_single_segments(bfs):
    # one call over 5 segments equals five single-segment calls bitwise, and matches the oracle
    n = 4096
    rng = np.random.default_rng(11)
    ys = rng.standard_normal((5, n)).astype(np.float32)
    temps = rng.standard_normal((7, 300))
    kappa = 3.0
    with bfs.Plan(n, 4096.0, kappa=kappa, templates=temps, precision="f32") as plan:
        with plan.filter(_dev(ys, np.float32)) as job:
            tb, _ = job.fetch_tails()
            sb = job.fetch_sigma()
        singles, ss = [], []
        for s in range(5):
            with plan.filter(_dev(ys[s], np.float32)) as job:
                t, _ = job.fetch_tails()
                t["segment"] = s
                singles.append(t)
                ss.append(job.fetch_sigma()[0])
    assert np.array_equal(np.concatenate(singles), tb)
    assert np.array_equal(np.stack(ss), sb)
    tw = [t.astype(np.float32).astype(np.float64) for t in temps]
    out = oracle.search([y.astype(np.float64) for y in ys], tw, kappa)
    compare_tails(tb, out["tails"], out["sigma"], kappa, TOL["f32"],
                  lambda s, j: oracle.correlate_fft(ys[s].astype(np.float64), tw[j]))


def test_repeated_runs_are_bitwise_identical(bfs):
    w = get_workload("C2")
    y, _ = make_segment(w, 0)
    grid = bfs.Grid(64, 16, w.f0_range, w.fdot_range, w.taus)
    with bfs.Plan(w.n, w.fs, kappa=4.0, grid=grid, precision="f32") as plan:
        res = []
        for _ in range(2):
            with plan.filter(_dev(y, np.float32)) as job:
                res.append((job.fetch_tails()[0], job.fetch_sigma()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert len(res[0][0]) > 0


def _c4_segments(count):
    w = get_workload("C4")
    segs = [make_segment(w, s)[0] for s in range(count)]
    return w, segs


def test_uneven_segments_in_one_call_match_oracle_and_single_calls(bfs):
    # batching form: segments of 2^14..2^17 samples in one filter call, grouped by length on the
    # device; every result equals the oracle and equals the same segment filtered alone (bitwise)
    w, segs = _c4_segments(6)
    lens = [len(y) for y in segs]
    assert len(set(lens)) >= 3, lens
    grid = bfs.Grid(8, 8, w.f0_range, w.fdot_range, w.taus)
    f0 = np.repeat(np.linspace(*w.f0_range, 8), 8)
    fd = np.tile(np.linspace(*w.fdot_range, 8), 8)
    tau = np.array([w.taus[j % len(w.taus)] for j in range(64)])
    temps = oracle.template_bank(f0, fd, tau, w.fs)
    flat = np.concatenate(segs).astype(np.float32)
    with bfs.Plan(1 << 17, w.fs, kappa=w.kappa, grid=grid, precision="f32", n_min=1 << 14) as plan:
        with plan.filter(torch.from_numpy(flat).cuda(), lengths=lens) as job:
            tails, total = job.fetch_tails()
            sig = job.fetch_sigma()
        alone_t, alone_s = [], []
        for s, y in enumerate(segs):
            with plan.filter(_dev(y, np.float32), lengths=[len(y)]) as job:
                t, _ = job.fetch_tails()
                t["segment"] = s
                alone_t.append(t)
                alone_s.append(job.fetch_sigma()[0])
    assert total == len(tails)
    assert np.array_equal(np.concatenate(alone_t), tails)
    assert np.array_equal(np.stack(alone_s), sig)
    out = oracle.search([y.astype(np.float64) for y in segs], temps, w.kappa)
    floor = np.array([[sigma_floor(t, y) for t in temps] for y in segs])
    assert np.max(np.abs(sig - out["sigma"]) / tol_scale(out["sigma"], floor)) <= TOL["f32"]
    common, band = compare_tails(tails, out["tails"], out["sigma"], w.kappa, TOL["f32"],
                                 lambda s, j: oracle.correlate_fft(segs[s].astype(np.float64), temps[j]), floor)
    print(f"uneven: {total} tails, common {common}, band-only {band}, lengths {lens}")
    assert common >= 0.99 * len(out["tails"])


def test_segment_offsets_select_the_samples(bfs):
    # segments read at arbitrary element offsets give the packed call's results bitwise
    n = 4096
    rng = np.random.default_rng(12)
    ys = rng.standard_normal((3, n)).astype(np.float32)
    buf = np.zeros(5 * n + 123, np.float32)
    offs = [4 * n + 100, 17, 2 * n + 5]
    for s, o in enumerate(offs):
        buf[o:o + n] = ys[s]
    temps = rng.standard_normal((5, 200))
    with bfs.Plan(n, 4096.0, kappa=2.5, templates=temps, precision="f32") as plan:
        with plan.filter(_dev(ys, np.float32)) as job:
            t0, s0 = job.fetch_tails()[0], job.fetch_sigma()
        with plan.filter(torch.from_numpy(buf).cuda(), lengths=[n] * 3, offsets=offs) as job:
            t1, s1 = job.fetch_tails()[0], job.fetch_sigma()
    assert len(t0) > 0 and np.array_equal(t0, t1) and np.array_equal(s0, s1)


def test_graph_replays_match_eager(bfs):
    # a graph plan captures the job once per shape and replays it; every replay (new data each
    # time, eager torch work and host syncs in between) equals the eager plan bitwise
    w, segs = _c4_segments(4)
    lens = [len(y) for y in segs]
    temps = np.random.default_rng(13).standard_normal((16, 2048))
    eager = bfs.Plan(1 << 17, w.fs, kappa=4.0, templates=temps, precision="f32", n_min=1 << 14)
    graph = bfs.Plan(1 << 17, w.fs, kappa=4.0, templates=temps, precision="f32", n_min=1 << 14, graph=True)
    try:
        for rep in range(4):
            flat = torch.from_numpy(np.concatenate(segs).astype(np.float32) * (1.0 + rep)).cuda()
            _ = torch.randn(1 << 20, device="cuda").sum().item()  # eager work between replays
            with eager.filter(flat, lengths=lens) as je, graph.filter(flat, lengths=lens) as jg:
                te, se = je.fetch_tails()[0], je.fetch_sigma()
                tg, sg = jg.fetch_tails()[0], jg.fetch_sigma()
            assert len(te) > 0 and np.array_equal(te, tg) and np.array_equal(se, sg), rep
    finally:
        eager.close()
        graph.close()


CANDIDATE_SIZES = [1 << 13, 1 << 14, 1 << 16, 1 << 17]


@pytest.mark.parametrize("n", CANDIDATE_SIZES, ids=[f"N{n}" for n in CANDIDATE_SIZES])
def test_every_kernel_candidate_matches_oracle(bfs, n):
    # the autotuner may pick any candidate: each one is held to the FP32 bar on its own
    rng = np.random.default_rng(n + 7)
    y = (rng.standard_normal(n) + 0.25).astype(np.float32)
    temps = [rng.standard_normal(l) for l in (1, 33, n // 4, n)]
    bank = np.zeros((len(temps), n))
    for j, w in enumerate(temps):
        bank[j, :len(w)] = w
    rho_o, sig_o = _oracle_dense([y.astype(np.float64)], [b.astype(np.float32).astype(np.float64) for b in bank])
    with bfs.Plan(n, 4096.0, kappa=5.0, templates=bank, precision="f32") as plan:
        count = plan.kernel_info()["n_candidates"]
    assert count >= 2
    for c in range(1, count + 1):
        with bfs.Plan(n, 4096.0, kappa=5.0, templates=bank, precision="f32", candidate=c) as plan:
            info = plan.kernel_info()
            assert info["candidate"] == c - 1
            rho_g, sig_g = plan.correlate_dense(_dev(y, np.float32))
            rho_g, sig_g = rho_g.cpu().numpy(), sig_g.cpu().numpy()
        err = max_rel_err(rho_g[0], rho_o[0], sig_o[0])
        print(f"N={n} candidate {info}: max err / sigma = {err:.3e}")
        assert err <= TOL["f32"] and np.max(np.abs(sig_g - sig_o) / sig_o) <= TOL["f32"]


def test_autotuned_plan_reports_timings_and_stays_correct(bfs):
    w = get_workload("C2")
    with bfs.Plan(1 << 14, w.fs, kappa=4.5, grid=bfs.Grid(32, 16, w.f0_range, w.fdot_range, (0.5,)),
                  precision="f32", n_min=1 << 13, autotune=True) as plan:
        for n in (1 << 13, 1 << 14):
            info = plan.kernel_info(n)
            print("autotuned", info)
            assert len(info["tuned_us"]) == info["n_candidates"] and all(t > 0 for t in info["tuned_us"])
            assert info["tuned_us"][info["candidate"]] == min(info["tuned_us"])
            tus = info["tile_us"]
            assert all(v > 0 for v in tus.values())
            # the largest tile within 2 % of the fastest (a little slack for float rounding)
            best = min(tus.values())
            assert tus[info["tile"]] <= 1.02 * best * (1 + 1e-5)
            assert all(us > 1.02 * best * (1 - 1e-5) for t, us in tus.items() if t > info["tile"])


@pytest.mark.parametrize("prec", ["f32-w16f", "f32-w16b"], ids=["fp16", "bf16"])
def test_c3_full_dense_bank_16bit_against_oracle_subset(bfs, prec):
    # C3: the C2 segment against all 1,048,576 chirps with 16-bit spectra resident (128 GiB);
    # templates 0..4095 against the FP64 oracle: every rho (dense), sigma and the tails.  FP16 is
    # held to 2e-3 sigma; BF16 to its error model's bound (it misses 2e-3, reported)
    w = get_workload("C3")
    y, _ = make_segment(w, 0)
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    f0, fd, tau = w.template_params()
    ids = np.arange(4096)
    temps = oracle.template_bank(f0, fd, tau, w.fs, ids=ids)
    out = oracle.search([y.astype(np.float64)], temps, w.kappa)
    floor = np.array([[sigma_floor(t, y) for t in temps]])
    bound = TOL[prec] if prec == "f32-w16f" else BF16_MODEL_BOUND
    with bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision=prec, tail_capacity=1 << 22) as plan:
        assert plan.k == 1 << 20 and plan.bank_bytes == (1 << 20) * (w.n // 2) * 4
        y_dev = _dev(y, np.float32)
        with plan.filter(y_dev) as job:
            tails, total = job.fetch_tails()
            sig = job.fetch_sigma()[:, :4096]
        err, sg, so = _dense_blocks(plan, y_dev, y.astype(np.float64), temps)
    rep = strict_report(err, so, floor[0])
    print(f"C3 {prec} dense rho, templates 0..4095: {rep}")
    assert np.array_equal(sg, sig[0])
    assert np.max(np.abs(sig - out["sigma"]) / tol_scale(out["sigma"], floor)) <= TOL[prec]
    assert rep["strict_max_err_over_sigma"] <= bound
    assert np.all(err <= bound * tol_scale(so, floor[0]))
    sub = tails[tails["template"] < 4096]
    common, band = compare_tails(sub, out["tails"], out["sigma"], w.kappa, bound,
                                 lambda s, j: oracle.correlate_fft(y.astype(np.float64), temps[j]), floor)
    print(f"C3 {prec}: {total} tails over 2^20 templates; subset common {common}, band-only {band}")


def test_workgroup_order_tiles_cover_every_correlation_once(bfs):
    # the XCD-aware order maps a 1-D grid onto (template, segment) pairs; K = 13 (not a
    # multiple of 8) and S = 7 (not a multiple of most tiles): every tile gives the same
    # sigma and tails as tile 1, bitwise, and those match the oracle
    n = 2048
    rng = np.random.default_rng(14)
    ys = rng.standard_normal((7, n)).astype(np.float32)
    temps = rng.standard_normal((13, 300))
    kappa = 3.0
    res = {}
    for t in (1, 2, 3, 4, 7, 16):
        with bfs.Plan(n, 4096.0, kappa=kappa, templates=temps, precision="f32", tile=t) as plan:
            assert plan.kernel_info()["tile"] == t
            with plan.filter(_dev(ys, np.float32)) as job:
                res[t] = (job.fetch_tails()[0], job.fetch_sigma())
    for t, (tl, sg) in res.items():
        assert np.array_equal(tl, res[1][0]) and np.array_equal(sg, res[1][1]), t
    tw = [x.astype(np.float32).astype(np.float64) for x in temps]
    out = oracle.search([y.astype(np.float64) for y in ys], tw, kappa)
    assert np.all(res[1][1] > 0) and np.max(np.abs(res[1][1] - out["sigma"]) / out["sigma"]) <= TOL["f32"]
    compare_tails(res[1][0], out["tails"], out["sigma"], kappa, TOL["f32"],
                  lambda s, j: oracle.correlate_fft(ys[s].astype(np.float64), tw[j]))


def test_persistent_kernel_with_tiles_and_a_ragged_bank(bfs):
    # the looping 2^16 kernels walk the tile order with a stride of their grid: with
    # K = 13 (three of the eight XCD residues hold one template fewer, so their workgroups
    # run out of items first) and S = 5 segments, every tile gives the same sigma and
    # tails as tile 1, bitwise, and those match the oracle
    n = 1 << 16
    rng = np.random.default_rng(16)
    ys = (rng.standard_normal((5, n)) + 0.1).astype(np.float32)
    temps = rng.standard_normal((13, 4096))
    kappa = 4.0
    with bfs.Plan(n, 4096.0, kappa=kappa, templates=temps, precision="f32") as plan:
        count = plan.kernel_info()["n_candidates"]
    looping = []
    for c in range(1, count + 1):
        with bfs.Plan(n, 4096.0, kappa=kappa, templates=temps, precision="f32", candidate=c) as plan:
            if plan.kernel_info()["loop"]:
                looping.append(c)
    assert looping, "no looping candidate at 2^16"
    tw = [x.astype(np.float32).astype(np.float64) for x in temps]
    out = oracle.search([y.astype(np.float64) for y in ys], tw, kappa)
    for c in looping:
        res = {}
        for t in (1, 2, 5):
            with bfs.Plan(n, 4096.0, kappa=kappa, templates=temps, precision="f32", candidate=c, tile=t) as plan:
                info = plan.kernel_info()
                assert info["loop"] and info["tile"] == t
                with plan.filter(_dev(ys, np.float32)) as job:
                    res[t] = (job.fetch_tails()[0], job.fetch_sigma())
        for t, (tl, sg) in res.items():
            assert np.array_equal(tl, res[1][0]) and np.array_equal(sg, res[1][1]), (c, t)
        assert np.max(np.abs(res[1][1] - out["sigma"]) / out["sigma"]) <= TOL["f32"]
        common, _ = compare_tails(res[1][0], out["tails"], out["sigma"], kappa, TOL["f32"],
                                  lambda s, j: oracle.correlate_fft(ys[s].astype(np.float64), tw[j]))
        print(f"looping candidate {c}: {len(res[1][0])} tails, {common} common with the oracle")
        assert common > 0


def test_split_kernel_with_tiles_and_a_ragged_bank(bfs):
    # the 2^17 correlations run as two halves with the even one waiting in scratch memory:
    # every candidate and tile over K = 13 templates and S = 3 segments gives tile 1's sigma
    # and tails bitwise, and those match the oracle
    n = 1 << 17
    rng = np.random.default_rng(17)
    ys = (rng.standard_normal((3, n)) + 0.1).astype(np.float32)
    temps = rng.standard_normal((13, 4096))
    kappa = 4.0
    with bfs.Plan(n, 4096.0, kappa=kappa, templates=temps, precision="f32") as plan:
        count = plan.kernel_info()["n_candidates"]
        assert plan.kernel_info()["split"]
    tw = [x.astype(np.float32).astype(np.float64) for x in temps]
    out = oracle.search([y.astype(np.float64) for y in ys], tw, kappa)
    ref = None
    for c in range(1, count + 1):
        for t in (1, 2, 3):
            with bfs.Plan(n, 4096.0, kappa=kappa, templates=temps, precision="f32", candidate=c, tile=t) as plan:
                assert plan.kernel_info()["tile"] == t
                with plan.filter(_dev(ys, np.float32)) as job:
                    got = (job.fetch_tails()[0], job.fetch_sigma())
            if t == 1:
                ref = got
                assert np.max(np.abs(got[1] - out["sigma"]) / out["sigma"]) <= TOL["f32"]
                common, _ = compare_tails(got[0], out["tails"], out["sigma"], kappa, TOL["f32"],
                                          lambda s, j: oracle.correlate_fft(ys[s].astype(np.float64), tw[j]))
                print(f"split candidate {c}: {len(got[0])} tails, {common} common with the oracle")
                assert common > 0
            else:
                assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (c, t)


def test_time_symmetric_bank_spectra_and_c1_search(bfs):
    # time-symmetric templates (chirp plus its reversal) synthesised on the device: spectra at
    # every plan length against the oracle, and the C1 search in FP64 against the oracle
    w = get_workload("C4")
    grid = bfs.Grid(4, 4, w.f0_range, w.fdot_range, w.taus, symmetric=True)
    f0 = np.repeat(np.linspace(*w.f0_range, 4), 4)
    fd = np.tile(np.linspace(*w.fdot_range, 4), 4)
    tau = np.array([w.taus[j % len(w.taus)] for j in range(16)])
    temps = oracle.template_bank(f0, fd, tau, w.fs, symmetric=True)
    with bfs.Plan(1 << 17, w.fs, kappa=5.0, grid=grid, precision="f32", n_min=1 << 14) as plan:
        for n in (1 << 14, 1 << 17):
            spec = plan.spectra(n=n).cpu().numpy()
            ref = np.fft.rfft(np.array([np.pad(t, (0, n - len(t))) for t in temps]), axis=-1)
            assert max_rel_err(spec, ref, np.max(np.abs(ref), axis=-1)) <= 2e-6, n
    c1 = get_workload("C1")
    y, _ = make_segment(c1, 0)
    g1 = bfs.Grid(c1.n_f0, c1.n_fdot, c1.f0_range, c1.fdot_range, c1.taus, symmetric=True)
    with bfs.Plan(c1.n, c1.fs, kappa=c1.kappa, grid=g1, precision="f64") as plan:
        with plan.filter(_dev(y, np.float64)) as job:
            tails, _ = job.fetch_tails()
            sig = job.fetch_sigma()
    f0, fd, tau = c1.template_params()
    bank = oracle.template_bank(f0, fd, tau, c1.fs, symmetric=True)
    out = oracle.search([y], bank, c1.kappa, keep_rho=True)
    assert np.max(np.abs(sig - out["sigma"]) / out["sigma"]) <= TOL["f64"]
    common, band = compare_tails(tails, out["tails"], out["sigma"], c1.kappa, TOL["f64"],
                                 lambda s, j: out["rho"][s][j])
    assert common > 50 and band <= 2


def test_band_threshold_matches_oracle(bfs):
    # finite band kappa sigma < |rho| < kappa_hi sigma (deep-search form) on the C2 segment
    w = get_workload("C2")
    y, _ = make_segment(w, 0)
    kappa, kappa_hi = 3.0, 3.5
    grid = bfs.Grid(16, 16, w.f0_range, w.fdot_range, w.taus)
    f0 = np.repeat(np.linspace(*w.f0_range, 16), 16)
    fd = np.tile(np.linspace(*w.fdot_range, 16), 16)
    temps = oracle.template_bank(f0, fd, np.full(256, 1.0), w.fs)
    with bfs.Plan(w.n, w.fs, kappa=kappa, kappa_hi=kappa_hi, grid=grid, precision="f32",
                  tail_capacity=1 << 22) as plan:
        with plan.filter(_dev(y, np.float32)) as job:
            tails, total = job.fetch_tails()
    out = oracle.search([y.astype(np.float64)], temps, kappa, kappa_hi=kappa_hi)
    sig = out["sigma"][0]
    floor = np.array([sigma_floor(t, y) for t in temps])
    tol = TOL["f32"] * tol_scale(sig, floor) / sig  # in units of sigma
    g = {(int(j), int(n)): float(r) for j, n, r in zip(tails["template"], tails["lag"], tails["rho"])}
    o = {(int(j), int(n)): float(r) for j, n, r in zip(out["tails"]["template"], out["tails"]["lag"], out["tails"]["rho"])}
    rows = {}

    def near_edge(j, n):
        if j not in rows:
            rows[j] = oracle.correlate_fft(y.astype(np.float64), temps[j]) / sig[j]
        a = abs(rows[j][n])
        return min(abs(a - kappa), abs(a - kappa_hi)) <= tol[j]

    only = (g.keys() - o.keys()) | (o.keys() - g.keys())
    assert all(near_edge(j, n) for j, n in only)
    assert all(abs(g[k] - o[k]) <= TOL["f32"] * tol_scale(sig[k[0]], floor[k[0]]) for k in g.keys() & o.keys())
    # every GPU tail inside the band, up to the tolerance at either edge (a GPU decision at
    # kappa sigma in FP32 can fall a rounding error on the other side of the oracle's)
    bad = [(j, n, abs(r) / sig[j], tol[j]) for (j, n), r in g.items()
           if not (kappa - tol[j] < abs(r) / sig[j] < kappa_hi + tol[j])]
    assert not bad, bad[:10]
    print(f"band: {total} GPU tails, {len(o)} oracle, {len(only)} differ within the band edges")
    assert len(g.keys() & o.keys()) > 1000 and len(only) <= len(o) // 100


def test_many_tails_come_back_complete_and_sorted(bfs):
    # kappa = 0 on 3 segments x 5 templates x 4096 lags: 61,440 tails, all written by the
    # wave-aggregated compaction and returned in (segment, template, lag) order
    n, S, K = 4096, 3, 5
    rng = np.random.default_rng(15)
    ys = rng.standard_normal((S, n)).astype(np.float32)
    temps = rng.standard_normal((K, 300))
    with bfs.Plan(n, 4096.0, kappa=0.0, templates=temps, precision="f32", tail_capacity=S * K * n) as plan:
        with plan.filter(_dev(ys, np.float32)) as job:
            tails, total = job.fetch_tails()
        rho, _ = plan.correlate_dense(_dev(ys, np.float32))
        rho = rho.cpu().numpy()
    assert total == S * K * n == len(tails)
    assert np.array_equal(tails["segment"], np.repeat(np.arange(S), K * n))
    assert np.array_equal(tails["template"], np.tile(np.repeat(np.arange(K), n), S))
    assert np.array_equal(tails["lag"], np.tile(np.arange(n), S * K))
    assert np.array_equal(tails["rho"].astype(np.float32), rho.reshape(-1))


def test_device_and_host_tail_sorts_agree(bfs):
    # 61,440 tails are ordered on the device; under an HBM budget with no room for the
    # device sort's work area the same fetch falls back to the host sort: same records
    n, S, K = 4096, 3, 5
    rng = np.random.default_rng(16)
    ys = _dev(rng.standard_normal((S, n)).astype(np.float32), np.float32)
    temps = rng.standard_normal((K, 300))
    kw = dict(kappa=0.0, templates=temps, precision="f32", tail_capacity=S * K * n)
    with bfs.Plan(n, 4096.0, **kw) as plan:
        need = plan.plan_bytes + plan.job_bytes([n] * S)
        with plan.filter(ys) as job:
            dev_sorted, total = job.fetch_tails()
    with bfs.Plan(n, 4096.0, hbm_budget_bytes=need + (256 << 10), **kw) as plan:
        with plan.filter(ys) as job:
            host_sorted, total2 = job.fetch_tails()
    assert total == total2 == S * K * n
    assert np.array_equal(dev_sorted, host_sorted)
