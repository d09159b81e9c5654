"""GPU: bfsearch_filter_noalloc against bfsearch_filter on the same inputs.

The no-allocation entry point runs the same kernels as bfsearch_filter with
the segment spectra in the library's fixed scratch area; its unsorted device
tail list, count and sigma must equal the sorted tails and sigma of the
ordinary call exactly.  Two calls in a row, the second with fewer segments,
check that the shared scratch area and the count start clean.
"""
import os

import numpy as np
import pytest

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


def _segments(n, count, dtype, seed):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((count, n)).astype(dtype))


def _key(t):
    return np.lexsort((t["lag"], t["template"], t["segment"]))


CASES = [("f32", 1 << 14, "", (5, 3)), ("f32", 1 << 16, "", (3, 1)), ("f32", 1 << 17, "", (4, 2)),
         ("f64", 1 << 13, "", (3, 2)), ("f64", 1 << 14, "", (2, 1)),
         ("f32", 1 << 14, "pairs", (4, 2)), ("f32", 1 << 16, "fused", (2, 1))]


@pytest.mark.parametrize("prec,n,form,counts", CASES, ids=[f"{p}-N{n}{'-' + f if f else ''}" for p, n, f, _ in CASES])
def test_noalloc_matches_filter(bfs, prec, n, form, counts):
    pairs = form == "pairs"
    grid = bfs.Grid(16, 16, (350.0, 2000.0), (-500.0, 500.0), (min(1.0, n / 4096.0 / 2),))
    dtype = np.float64 if prec == "f64" else np.float32
    tdt = torch.float64 if prec == "f64" else torch.float32
    cap = 1 << 18
    with bfs.Plan(n, 4096.0, kappa=4.0, grid=grid, precision=prec, tail_capacity=cap, pairs=pairs,
                  fused=form == "fused") as plan:
        tails_buf = torch.empty(cap * plan.tail_dtype.itemsize, dtype=torch.uint8, device="cuda:0")
        count = torch.empty(1, dtype=torch.int64, device="cuda:0")
        for call, S in enumerate(counts):
            y = _segments(n, S, dtype, seed=1000 * call + n + (7 if pairs else 0))
            y_dev = torch.from_numpy(y).to("cuda:0", dtype=tdt)
            sigma = torch.full((S, plan.k), -1.0, dtype=torch.float64, device="cuda:0")
            print(f"noalloc call {call}: {prec} N={n} S={S} pairs={pairs}", flush=True)
            plan.filter_noalloc(y_dev, tails_buf, count, sigma)
            torch.cuda.synchronize()
            total = int(count.item())
            got = bfs.tails_from_device(tails_buf, total, plan.tail_dtype)
            got = got[_key(got)]
            with plan.filter(y_dev) as job:
                want, want_total = job.fetch_tails()
                want_sigma = job.fetch_sigma()
            assert total == want_total and total == len(got)
            assert total > 0
            for f in ("segment", "template", "lag"):
                np.testing.assert_array_equal(got[f], want[f])
            np.testing.assert_array_equal(got["rho"], want["rho"])
            np.testing.assert_array_equal(sigma.cpu().numpy(), want_sigma)


def test_noalloc_rejects_what_does_not_fit(bfs):
    n = 1 << 16
    grid = bfs.Grid(2, 2, (350.0, 2000.0), (-500.0, 500.0), (1.0,))
    with bfs.Plan(n, 4096.0, kappa=5.0, grid=grid, precision="f32") as plan:
        # FP32 spectra take 4 bytes per sample, and the segment transform a scratch of that size
        s_max = bfs.NOALLOC_SCRATCH_BYTES // (2 * n * 4)
        y = torch.zeros((s_max + 1, n), dtype=torch.float32, device="cuda:0")
        tails_buf = torch.empty(16 * plan.tail_dtype.itemsize, dtype=torch.uint8, device="cuda:0")
        count = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        with pytest.raises(bfs.BfsError) as e:
            plan.filter_noalloc(y, tails_buf, count)
        assert e.value.status == bfs.BFS_ERR_SCRATCH_LIMIT
        plan.filter_noalloc(y[:s_max], tails_buf, count)  # the largest batch that fits
        torch.cuda.synchronize()
        assert int(count.item()) == 0  # zero segments: zero sigma, no tails
    with bfs.Plan(1 << 14, 4096.0, kappa=5.0, grid=grid, precision="f32", project=True) as plan:
        y = torch.zeros((1, 1 << 14), dtype=torch.float32, device="cuda:0")
        with pytest.raises(bfs.BfsError) as e:
            plan.filter_noalloc(y, tails_buf, count)
        assert e.value.status == bfs.BFS_ERR_INVALID_ARG
