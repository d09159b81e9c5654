"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something it cannot simply restate:
a brute-force sum, a closed form, an identity, a library special case or a
Gaussian expectation.  The comment on each test names the plausible mistake
it would catch.
"""
import math
import os

import numpy as np
import pytest
import scipy.signal
import scipy.special

import oracle
from synthetic import bandlimited_noise, seeded_rng, unit_hann_chirp, get_workload, make_segment


def _rng(seed):
    return np.random.default_rng(seed)


def _brute_force(y, w):
    """Pure-Python circular correlation: rho[n] = sum_m w[m] y[(n+m) % N]."""
    n = len(y)
    out = []
    for lag in range(n):
        acc = 0.0
        for m in range(len(w)):
            acc += w[m] * y[(lag + m) % n]
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("n,l", [(8, 1), (8, 3), (8, 8), (16, 4), (16, 16), (64, 1), (64, 16), (64, 64),
                                 (256, 3), (256, 64), (1024, 1), (1024, 3), (1024, 256)])
def test_fft_and_direct_match_brute_force(n, l):
    # catches: conj on the wrong operand, a wrong irfft normalisation, a shifted or reversed lag
    r = _rng(1000 * n + l)
    y = r.standard_normal(n)
    w = r.standard_normal(l)
    ref = _brute_force(list(y), list(w))
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(oracle.correlate_fft(y, w) - ref)) <= 1e-12 * scale
    assert np.max(np.abs(oracle.correlate_direct(y, w) - ref)) <= 1e-12 * scale


@pytest.mark.parametrize("n0", [0, 5, 1023])
def test_impulse_closed_form(n0):
    # y = delta at n0  =>  rho[n] = w[(n0 - n) mod N]; catches a lag sign error
    n, l = 1024, 100
    w = _rng(7).standard_normal(l)
    y = np.zeros(n)
    y[n0] = 1.0
    wpad = np.zeros(n)
    wpad[:l] = w
    expect = wpad[(n0 - np.arange(n)) % n]
    np.testing.assert_allclose(oracle.correlate_fft(y, w), expect, rtol=0, atol=1e-13)


@pytest.mark.parametrize("q,l,phi", [(3, 100, 0.0), (37, 1000, 0.7), (200, 4096, -1.1)])
def test_rectangular_template_tone_closed_form(q, l, phi):
    # w = 1 on L samples, y = cos(2 pi q n / N + phi): Dirichlet-kernel closed form
    n = 8192
    y = np.cos(2 * np.pi * q * np.arange(n) / n + phi)
    w = np.ones(l)
    k = np.arange(n)
    amp = math.sin(math.pi * q * l / n) / math.sin(math.pi * q / n)
    expect = amp * np.cos(2 * np.pi * q * k / n + phi + math.pi * q * (l - 1) / n)
    np.testing.assert_allclose(oracle.correlate_fft(y, w), expect, rtol=0, atol=1e-9 * abs(amp) + 1e-10)


def test_parseval_identity_any_input():
    # Eq. (6) time domain == its exact Parseval form for any real input, including DC and Nyquist power
    r = _rng(3)
    n = 4096
    for trial in range(5):
        y = r.standard_normal(n) + (0.3 if trial % 2 else 0.0)
        w = r.standard_normal(300)
        rho = oracle.correlate_fft(y, w)
        c = np.fft.rfft(rho)
        st = oracle.sigma_time(rho)
        sf = oracle.sigma_parseval(c, n)
        assert abs(st - sf) <= 1e-12 * st
        # the naive time-domain RMS, written out
        assert abs(st - math.sqrt(sum(v * v for v in rho) / n)) <= 1e-12 * st


def test_eq7_equals_parseval_for_bandlimited_only():
    # the paper's sqrt(2)/N form omits C_0 and C_{N/2}: exact for band-limited data, biased otherwise
    n, fs = 8192, 4096.0
    y = bandlimited_noise(n, fs, seeded_rng(99, 0, 0, "noise"))
    w = oracle.chirp_template(800.0, 100.0, 1024, fs)
    rho = oracle.correlate_fft(y, w)
    c = np.fft.rfft(rho)
    assert abs(oracle.sigma_eq7(c, n) - oracle.sigma_parseval(c, n)) <= 1e-12 * oracle.sigma_parseval(c, n)
    y2 = y + 0.5  # DC offset: C_0 != 0
    rho2 = oracle.correlate_fft(y2, np.ones(64))
    c2 = np.fft.rfft(rho2)
    assert oracle.sigma_eq7(c2, n) < 0.9 * oracle.sigma_parseval(c2, n)
    assert abs(oracle.sigma_parseval(c2, n) - oracle.sigma_time(rho2)) <= 1e-12 * oracle.sigma_time(rho2)


def test_sigma_expectation_equals_inband_template_energy():
    # E[sigma^2] over band-limited unit noise = (1/N) sum_{k in band} |W_k|^2 (full spectrum);
    # catches a wrong 1/N or a factor 2 in sigma.  Template straddles the 350 Hz edge.
    n, fs = 4096, 4096.0
    w = oracle.chirp_template(250.0, 800.0, 1024, fs)  # 250 -> 450 Hz over 0.25 s
    wk = np.fft.fft(np.concatenate([w, np.zeros(n - len(w))]))
    f = np.abs(np.fft.fftfreq(n, d=1.0 / fs))
    band = (f >= 350.0) & (f <= 2000.0) & (f > 0) & (f < fs / 2)
    expect = np.sum(np.abs(wk[band]) ** 2) / n
    assert 0.2 < expect < 0.9
    vals = []
    for s in range(400):
        y = bandlimited_noise(n, fs, seeded_rng(77, 0, s, "noise"))
        vals.append(oracle.sigma_time(oracle.correlate_fft(y, w)) ** 2)
    vals = np.array(vals)
    sem = vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(vals.mean() - expect) < 5 * sem + 1e-3 * expect


def test_gaussian_exceedance_fractions():
    # pooled P(|rho|/sigma > kappa) ~ erfc(kappa/sqrt 2) for band-limited Gaussian noise (Sec. 3).
    # Wide-band chirps keep the effective sample count high; dividing by the realised sigma of each
    # correlation still trims the far tail slightly, hence the looser bound at kappa = 3.
    n, fs = 8192, 4096.0
    templates = [oracle.chirp_template(f0, fd, 1024, fs) for f0 in (500.0, 900.0, 1300.0, 1700.0)
                 for fd in (-1600.0, 0.0, 1600.0)]
    counts = {1.0: 0, 2.0: 0, 3.0: 0}
    total = 0
    for s in range(64):
        y = bandlimited_noise(n, fs, seeded_rng(55, 0, s, "noise"))
        rho = oracle.correlate_fft(y, np.array(templates))
        z = np.abs(rho) / oracle.sigma_time(rho)[:, None]
        for k in counts:
            counts[k] += int(np.sum(z > k))
        total += z.size
    for k, c in counts.items():
        p = scipy.special.erfc(k / math.sqrt(2.0))
        tol = 0.05 if k < 3 else 0.20
        assert abs(c / total - p) <= tol * p, (k, c / total, p)


def test_hann_is_numpy_symmetric_hann():
    for l in (2, 3, 16, 1024, 4097):
        np.testing.assert_allclose(oracle.hann(l), np.hanning(l), rtol=0, atol=1e-15)
    assert oracle.hann(1).tolist() == [1.0]


def test_chirp_quarter_rate_tone_exact():
    # f0 = fs/4, fdot = 0, untapered: cos(pi m / 2) = 1, 0, -1, 0, ...
    w = oracle.chirp_template(1024.0, 0.0, 16, 4096.0, taper=False, normalize=False)
    np.testing.assert_allclose(w, np.tile([1.0, 0.0, -1.0, 0.0], 4), rtol=0, atol=1e-15)


@pytest.mark.parametrize("f0,fdot", [(600.0, 300.0), (1500.0, -400.0)])
def test_chirp_instantaneous_frequency(f0, fdot):
    # local frequency of the untapered chirp is f0 + fdot t (pins the 1/2 in the phase and fdot's sign)
    fs, l = 4096.0, 4096
    w = oracle.chirp_template(f0, fdot, l, fs, taper=False, normalize=False)
    ph = np.unwrap(np.angle(scipy.signal.hilbert(w)))
    finst = np.diff(ph) * fs / (2 * np.pi)
    t = (np.arange(l - 1) + 0.5) / fs
    mid = slice(200, l - 200)
    assert np.max(np.abs(finst[mid] - (f0 + fdot * t[mid]))) < 2.0


def test_template_unit_energy_and_grid_order():
    f0, fd, tau = oracle.grid_params(3, 4, (400.0, 800.0), (-100.0, 200.0), (0.5, 1.0))
    assert f0.tolist() == [400.0] * 4 + [600.0] * 4 + [800.0] * 4
    assert fd.tolist() == [-100.0, 0.0, 100.0, 200.0] * 3
    assert tau.tolist() == [0.5, 1.0] * 6
    for w in oracle.template_bank(f0, fd, tau, 4096.0):
        assert abs(np.dot(w, w) - 1.0) < 1e-13


def test_cauchy_schwarz_recovers_noise_free_injection():
    # y = A * (unit chirp of grid point j) at lag n0, no noise: the raw |rho| maximum over the
    # bank is A exactly, at (j, n0); the injected chirp is built by the input generator's own code.
    w = get_workload("C1")
    f0, fd, tau = w.template_params()
    bank = oracle.template_bank(f0, fd, tau, w.fs)
    n, amp, j_true, n0 = w.n, 7.5, 19, 3001
    y = np.zeros(n)
    s = unit_hann_chirp(f0[j_true], fd[j_true], int(round(tau[j_true] * w.fs)), w.fs)
    y[n0:n0 + len(s)] = amp * s
    rho = oracle.correlate_fft(y, np.array(bank))
    j, lag = np.unravel_index(np.argmax(np.abs(rho)), rho.shape)
    assert (j, lag) == (j_true, n0)
    assert abs(rho[j, lag] - amp) < 1e-12 * amp
    others = np.abs(np.delete(rho, j_true, axis=0))
    assert others.max() < amp * (1 - 1e-6)


def test_threshold_strict_and_absolute():
    sigma, kappa = 2.0, 3.0
    rho = np.array([6.0, -6.0, 6.0000001, -6.0000001, 5.9, -7.0, 0.0])
    assert oracle.threshold_tails(rho, sigma, kappa).tolist() == [2, 3, 5]
    assert oracle.threshold_tails(rho, 0.0, kappa).tolist() == []


def test_shift_equivariance_and_linearity():
    r = _rng(11)
    n = 2048
    y1, y2 = r.standard_normal(n), r.standard_normal(n)
    w = r.standard_normal(200)
    rho1 = oracle.correlate_fft(y1, w)
    np.testing.assert_allclose(oracle.correlate_fft(np.roll(y1, 37), w), np.roll(rho1, 37), atol=1e-11)
    np.testing.assert_allclose(oracle.correlate_fft(2.0 * y1 - 3.0 * y2, w),
                               2.0 * rho1 - 3.0 * oracle.correlate_fft(y2, w), atol=1e-11)


def test_search_tails_equal_brute_force_threshold():
    # the full search (batched FFT, sigma, strict threshold, sort) against brute force at tiny N
    r = _rng(5)
    segs = [r.standard_normal(64), r.standard_normal(64)]
    temps = [r.standard_normal(5), r.standard_normal(16), r.standard_normal(1)]
    kappa = 1.5
    out = oracle.search(segs, temps, kappa, keep_rho=True)
    expect = []
    for s, y in enumerate(segs):
        for j, w in enumerate(temps):
            rho = _brute_force(list(y), list(w))
            sig = math.sqrt(sum(v * v for v in rho) / len(rho))
            assert abs(out["sigma"][s, j] - sig) <= 1e-12 * sig
            assert abs(out["sigma_f"][s, j] - sig) <= 1e-12 * sig
            for lag, v in enumerate(rho):
                if abs(v) > kappa * sig:
                    expect.append((s, j, lag, v))
    got = out["tails"]
    assert [(int(a), int(b), int(c)) for a, b, c, _ in got] == [(a, b, c) for a, b, c, _ in expect]
    np.testing.assert_allclose(got["rho"], [e[3] for e in expect], rtol=1e-12, atol=1e-12)


def test_c1_injection_recovered_by_raw_rho():
    # C1: SNR-20 chirp (600 Hz, +50 Hz/s, 0.25 s) in band-limited noise; the raw-|rho| maximum
    # sits at f0 = 600 Hz with fdot on one of the two neighbouring grid values, near the offset
    w = get_workload("C1")
    y, inj = make_segment(w, 0)
    f0, fd, tau = w.template_params()
    bank = oracle.template_bank(f0, fd, tau, w.fs)
    out = oracle.search([y], bank, w.kappa, keep_rho=True)
    rho = out["rho"][0]
    noise_out = oracle.search([_noise_only(w)], bank, w.kappa)
    assert len(out["tails"]) > 50
    assert len(out["tails"]) > 2 * max(1, len(noise_out["tails"]))
    j, lag = np.unravel_index(np.argmax(np.abs(rho)), rho.shape)
    assert f0[j] == 600.0
    assert np.min(np.abs(fd[j] - np.array([200.0 / 7, 600.0 / 7]))) < 1e-9
    assert abs(int(lag) - inj[0].offset) <= 512


def _noise_only(w):
    return bandlimited_noise(w.n, w.fs, seeded_rng(w.config_id, 0, 0, "noise"))


def test_max_projection_equals_brute_force_argmax():
    # per-lag max projection (Sec. 3.3, Eqs. 13-17) against an explicit argmax over every
    # template's brute-force rho/sigma at each (segment, lag), lowest id first on ties
    r = _rng(21)
    segs = [r.standard_normal(64), r.standard_normal(32)]
    temps = [r.standard_normal(5), r.standard_normal(12), r.standard_normal(1), r.standard_normal(7)]
    kappa = 1.2
    out = oracle.search(segs, temps, kappa)
    proj = oracle.max_projection(out["tails"], out["sigma"])
    expect = []
    for s, y in enumerate(segs):
        rows = []
        for w in temps:
            rho = _brute_force(list(y), list(w))
            sig = math.sqrt(sum(v * v for v in rho) / len(rho))
            rows.append((rho, sig))
        for lag in range(len(y)):
            best = None
            for j, (rho, sig) in enumerate(rows):
                v = rho[lag] / sig
                if abs(rho[lag]) > kappa * sig and (best is None or abs(v) > abs(best[1])):
                    best = (j, v)
            if best is not None:
                expect.append((s, lag, best[0], best[1]))
    assert [(int(a), int(b), int(c)) for a, b, c, _ in proj] == [(a, b, c) for a, b, c, _ in expect]
    np.testing.assert_allclose(proj["snr"], [e[3] for e in expect], rtol=1e-11, atol=1e-12)
    assert len(proj) > 10


def test_max_projection_ties_scale_and_sign():
    r = _rng(22)
    y = r.standard_normal(128)
    w = r.standard_normal(9)
    # templates 1 and 3 are w scaled by 2 and 0.5: the same rho/sigma everywhere, so every lag
    # they win goes to template 1 (lowest id among the tied); template 0 is unrelated
    temps = [r.standard_normal(9), 2.0 * w, r.standard_normal(4), 0.5 * w]
    out = oracle.search([y], temps, 1.0)
    proj = oracle.max_projection(out["tails"], out["sigma"])
    assert 3 not in set(proj["template"].tolist()) and 1 in set(proj["template"].tolist())
    # a single template: the projection is its tail list, with snr = rho / sigma (sign kept)
    one = oracle.search([y], [w], 1.0)
    p1 = oracle.max_projection(one["tails"], one["sigma"])
    assert np.array_equal(p1["lag"], one["tails"]["lag"]) and np.all(p1["template"] == 0)
    np.testing.assert_allclose(p1["snr"], one["tails"]["rho"] / one["sigma"][0, 0], rtol=1e-14)
    assert np.any(p1["snr"] < 0) and np.any(p1["snr"] > 0)


def test_time_symmetric_template_mirrors_correlation_of_reversed_data():
    # a time-symmetric template (w[m] = w[L-1-m]) correlated with time-reversed data gives the
    # mirrored correlation: rho_rev[n] = rho[(-n - L) mod N]; a one-way chirp does not
    n, fs = 256, 4096.0
    ws = oracle.chirp_template(600.0, 900.0, 64, fs, symmetric=True)
    wf = oracle.chirp_template(600.0, 900.0, 64, fs)
    assert np.array_equal(ws, ws[::-1]) and abs(np.dot(ws, ws) - 1.0) < 1e-12
    y = _rng(23).standard_normal(n)
    yr = y[::-1].copy()
    mirror = (-np.arange(n) - len(ws)) % n
    np.testing.assert_allclose(oracle.correlate_fft(yr, ws), oracle.correlate_fft(y, ws)[mirror], atol=1e-12)
    assert not np.allclose(oracle.correlate_fft(yr, wf), oracle.correlate_fft(y, wf)[mirror], atol=1e-6)
    # it responds to the chirp and to its time reversal alike (ascending and descending searches)
    up = oracle.correlate_fft(np.pad(wf, (0, n - 64)), ws)[0]
    down = oracle.correlate_fft(np.pad(wf[::-1], (0, n - 64)), ws)[0]
    assert abs(up - down) < 1e-12 and up > 0.6


def test_band_threshold_keeps_only_the_band():
    r = _rng(24)
    rho = r.standard_normal(4000)
    sig = 1.0
    band = oracle.threshold_tails(rho, sig, 2.0, 2.5)
    expect = [i for i, v in enumerate(rho) if 2.0 < abs(v) < 2.5]
    assert band.tolist() == expect and len(expect) > 20
    # the open band equals the one-sided threshold minus the upper tail
    hi = oracle.threshold_tails(rho, sig, 2.5 - 1e-15)
    lo = oracle.threshold_tails(rho, sig, 2.0)
    assert sorted(set(lo.tolist()) - set(hi.tolist())) == expect
    # both edges strict: values exactly at kappa sigma or kappa_hi sigma are outside
    edges = np.array([2.5, -2.5, 2.0, 2.2, -2.3, -2.0])
    assert oracle.threshold_tails(edges, 1.0, 2.0, 2.5).tolist() == [3, 4]
    out = oracle.search([rho[:512]], [np.ones(1)], 1.5, kappa_hi=2.0)
    assert all(1.5 < abs(v) / out["sigma"][0, 0] < 2.0 for v in out["tails"]["rho"])


# ------------------------------------------------------------------ two detectors --

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table3_projection():
    """The rows of Table 3 as a projection of pair 0 (H1 = segment 0, L1 = segment 1): lags are
    offsets from the first printed row, each distinct printed frequency is one template."""
    rows = np.loadtxt(os.path.join(GOLDEN, "table3_b161_rows.txt"), comments="#")
    freqs = sorted({f for f in np.concatenate([rows[:, 3], rows[:, 4]]) if f > 0})
    tid = {f: i for i, f in enumerate(freqs)}
    recs = []
    for off, ra, rb, fa, fb in rows:
        lag = int(off - rows[0, 0])
        if ra > 0:
            recs.append((0, lag, tid[fa], ra / 1000.0))
        if rb > 0:
            recs.append((1, lag, tid[fb], rb / 1000.0))
    proj = np.array(recs, dtype=oracle.PEAK_DTYPE)
    return rows, proj, np.array(freqs, dtype=np.float64)


@pytest.mark.parametrize("delta,offsets", [
    (50.0, [17713196, 17713197, 17713198, 17713199]),  # the four simultaneous hits, all within 50 Hz
    (5.0, [17713197, 17713198, 17713199]),             # 497 vs 489 Hz is 8 Hz apart
    (1.5, [17713197, 17713198]),                       # 563 vs 565 Hz is 2 Hz apart
    (1.0, []),                                         # 1 Hz apart is not strictly within 1 Hz
])
def test_coincidences_of_table3_rows(delta, offsets):
    # pinned by the paper's printed output: the simultaneous hits of Table 3 are the rows with a
    # hit in both detectors; the frequency window keeps pairs strictly closer than delta.
    # catches: a missing abs, <= for <, comparing template ids instead of frequencies, a lag
    # or pair taken from one channel only
    rows, proj, f0 = _table3_projection()
    got = oracle.coincidences(proj, f0, delta)
    assert [int(rows[0, 0]) + int(n) for n in got["lag"]] == offsets
    assert np.all(got["pair"] == 0)
    by_off = {int(r[0]): r for r in rows}
    for c in got:
        r = by_off[int(rows[0, 0]) + int(c["lag"])]
        assert f0[c["template_a"]] == r[3] and f0[c["template_b"]] == r[4]
        assert c["snr_a"] == r[1] / 1000.0 and c["snr_b"] == r[2] / 1000.0


def _pair_search(n_pairs=2, n=2048, same=False, seed=40):
    w = get_workload("C1")
    f0, fd, tau = oracle.grid_params(6, 4, (400.0, 1800.0), (-200.0, 200.0), (0.125,))
    bank = oracle.template_bank(f0, fd, tau, w.fs)
    a = [bandlimited_noise(n, w.fs, seeded_rng(9, 0, p, "noise")) for p in range(n_pairs)]
    b = a if same else [bandlimited_noise(n, w.fs, seeded_rng(9, 1, p, "noise")) for p in range(n_pairs)]
    segs = oracle.pair_segments(a, b)
    out = oracle.search(segs, bank, 2.5)
    return oracle.max_projection(out["tails"], out["sigma"]), f0


def test_coincidences_of_identical_channels_are_every_projected_lag():
    # catches: a channel or pair index taken from the wrong segment, strict vs loose window
    proj, f0 = _pair_search(same=True)
    got = oracle.coincidences(proj, f0, 50.0)
    first = proj[proj["segment"] % 2 == 0]
    assert len(got) == len(first) > 0
    assert np.array_equal(got["pair"], first["segment"] // 2) and np.array_equal(got["lag"], first["lag"])
    assert np.array_equal(got["template_a"], got["template_b"]) and np.array_equal(got["snr_a"], got["snr_b"])
    assert len(oracle.coincidences(proj, f0, 0.0)) == 0  # |f_a - f_b| = 0 is not < 0


def test_coincidences_swap_symmetry_and_monotone_window():
    proj, f0 = _pair_search()
    swapped = proj.copy()
    swapped["segment"] = swapped["segment"] ^ 1
    wide = oracle.coincidences(proj, f0, np.inf)
    # an unbounded window leaves the simultaneous hits: lags present in both channels
    both = {(int(s) // 2, int(n)) for s, n in zip(proj["segment"], proj["lag"]) if s % 2 == 0} & \
           {(int(s) // 2, int(n)) for s, n in zip(proj["segment"], proj["lag"]) if s % 2 == 1}
    assert {(int(p), int(n)) for p, n in zip(wide["pair"], wide["lag"])} == both and len(both) > 0
    prev = None
    for delta in (0.0, 100.0, 300.0, 1000.0, np.inf):
        got = oracle.coincidences(proj, f0, delta)
        sw = oracle.coincidences(swapped, f0, delta)
        assert np.array_equal(got["lag"], sw["lag"]) and np.array_equal(got["template_a"], sw["template_b"])
        assert np.array_equal(got["snr_a"], sw["snr_b"])
        keys = {(int(p), int(n)) for p, n in zip(got["pair"], got["lag"])}
        assert prev is None or prev <= keys
        assert all(abs(f0[a] - f0[b]) < delta for a, b in zip(got["template_a"], got["template_b"]))
        prev = keys


def test_chirp_in_both_channels_gives_coincidences_at_its_offset():
    # one chirp injected at the same offset into two independent noise channels (Sec. 5: an
    # injection seen in both detectors): coincidences appear around the injected offset, and
    # there the winning templates of both channels are the injected chirp's neighbours in f0
    fs, n, L, off = 4096.0, 8192, 1024, 3000
    f0, fd, tau = oracle.grid_params(8, 8, (400.0, 1800.0), (-200.0, 200.0), (0.25,))
    bank = oracle.template_bank(f0, fd, tau, fs)
    s = 16.0 * unit_hann_chirp(600.0, 0.0, L, fs)
    a = bandlimited_noise(n, fs, seeded_rng(9, 0, 7, "noise"))
    b = bandlimited_noise(n, fs, seeded_rng(9, 1, 7, "noise"))
    a[off:off + L] += s
    b[off:off + L] += s
    out = oracle.search(oracle.pair_segments([a], [b]), bank, 4.0)
    proj = oracle.max_projection(out["tails"], out["sigma"])
    got = oracle.coincidences(proj, f0, 50.0)
    near = got[np.abs(got["lag"].astype(np.int64) - off) <= 64]
    assert len(near) > 0
    assert np.all(np.abs(f0[near["template_a"]] - 600.0) < 100.0)
    assert np.all(np.abs(f0[near["template_b"]] - 600.0) < 100.0)
    # no chirp in the second channel: far fewer coincidences near the offset
    b2 = bandlimited_noise(n, fs, seeded_rng(9, 1, 7, "noise"))
    out2 = oracle.search(oracle.pair_segments([a], [b2]), bank, 4.0)
    got2 = oracle.coincidences(oracle.max_projection(out2["tails"], out2["sigma"]), f0, 50.0)
    assert len(got2[np.abs(got2["lag"].astype(np.int64) - off) <= 64]) < len(near)
