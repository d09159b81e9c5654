"""Serving form on the GPU: continuous batching over several streams gives every request
exactly the result it gets alone, and the results match the oracle."""
import os

import numpy as np
import pytest

import oracle
from synthetic import get_workload
from tests.parity import TOL, compare_tails, sigma_floor, tol_scale

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


@pytest.mark.parametrize("prec", ["f32", "f32-w16f"])
def test_served_mix_equals_alone_and_oracle(bfs, prec):
    from paper_1708_01609_amd.serve import GpuExecutor, Request, serve
    from synthetic.strain import bandlimited_noise, seeded_rng

    w = get_workload("C5")
    lengths = (1 << 13, 1 << 14, 1 << 15)
    rng = np.random.default_rng(21)
    reqs = []
    for i in range(24):
        n = int(rng.choice(lengths))
        y = bandlimited_noise(n, w.fs, seeded_rng(99, i % 4, i, "noise")).astype(np.float32)
        # the first 15 arrive together (three full jobs of five), the rest trickle in
        reqs.append(Request(i, 0.0 if i < 15 else 0.002 * i, y, channel=i % 4))
    grid = bfs.Grid(16, 8, w.f0_range, w.fdot_range, (0.5,))
    kappa = 4.0
    with bfs.Plan(1 << 15, w.fs, kappa=kappa, grid=grid, precision=prec, n_min=1 << 13) as plan:
        ex = GpuExecutor(plan, slots=3, max_batch=5)
        budget = 3 * plan.job_bytes([1 << 15] * 5)
        st = serve(ex, reqs, slots=3, max_batch=5, budget_bytes=budget)
        assert len(st.results) == 24 and not st.rejected
        assert st.max_inflight_bytes <= budget
        mixed = [r for r in st.results.values() if r.batch > 1]
        assert mixed, "no request shared a job"
        for r in reqs:
            y = torch.from_numpy(r.samples).cuda()
            with plan.filter(y, lengths=[len(r.samples)]) as job:
                t, _ = job.fetch_tails()
                sg = job.fetch_sigma()[0]
            t["segment"] = r.rid
            got = st.results[r.rid]
            assert np.array_equal(got.tails, t), r.rid
            assert np.array_equal(got.sigma, sg), r.rid
    s = st.summary(128)
    print(f"{prec}: {s}")
    # oracle parity for a few requests of each length
    f0 = np.repeat(np.linspace(*w.f0_range, 16), 8)
    fd = np.tile(np.linspace(*w.fdot_range, 8), 16)
    temps = oracle.template_bank(f0, fd, np.full(128, 0.5), w.fs)
    for n in lengths:
        r = next(q for q in reqs if len(q.samples) == n)
        out = oracle.search([r.samples.astype(np.float64)], temps, kappa)
        got = st.results[r.rid]
        t = got.tails.copy()
        t["segment"] = 0
        floor = np.array([[sigma_floor(tm, r.samples) for tm in temps]])
        scale = tol_scale(out["sigma"][0], floor[0])
        assert np.max(np.abs(got.sigma - out["sigma"][0]) / scale) <= TOL[prec]
        compare_tails(t, out["tails"], out["sigma"], kappa, TOL[prec],
                      lambda s, j: oracle.correlate_fft(r.samples.astype(np.float64), temps[j]), floor)
