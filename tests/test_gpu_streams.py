"""Jobs queued from many caller streams at once: the segment transforms run on each caller's
stream, the fused kernels on the plan's paired streams (at most 16 are created; further
caller streams share them).  Every job must return what the same job returns alone."""
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


def test_twenty_caller_streams_match_one_stream(bfs):
    n, S = 4096, 2
    rng = np.random.default_rng(40)
    temps = rng.standard_normal((24, 300))
    ys = [torch.from_numpy(rng.standard_normal(S * n).astype(np.float32)).cuda() for _ in range(20)]
    with bfs.Plan(n, 4096.0, kappa=2.5, templates=temps, precision="f32") as plan:
        alone = []
        for y in ys:
            with plan.filter(y, lengths=[n] * S) as job:
                alone.append((job.fetch_tails()[0], job.fetch_sigma()))
        streams = [torch.cuda.Stream() for _ in ys]
        jobs = [plan.filter(y, lengths=[n] * S, stream=s) for y, s in zip(ys, streams)]  # all in flight
        for job, (tails, sigma) in zip(jobs, alone):
            t, total = job.fetch_tails()
            assert total == len(tails) > 0
            assert np.array_equal(t, tails)
            assert np.array_equal(job.fetch_sigma(), sigma)
            job.release()
