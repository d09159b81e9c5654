"""Error paths and degenerate inputs of the C ABI on the GPU (host-forced conditions only)."""
import os

import numpy as np
import pytest

import oracle
from tests.parity import TOL, compare_tails

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


def test_nan_segment_gives_nan_sigma_and_no_tails(bfs):
    n = 4096
    y = np.random.default_rng(30).standard_normal(n)
    y[123] = np.nan
    with bfs.Plan(n, 4096.0, kappa=1.0, templates=np.ones((3, 40)), precision="f32") as plan:
        with plan.filter(_dev(y)) as job:
            tails, total = job.fetch_tails()
            sig = job.fetch_sigma()
    assert total == 0 and np.all(np.isnan(sig))


def test_hbm_budget_limits_plan_and_jobs(bfs):
    n, K = 1 << 14, 64
    temps = np.random.default_rng(31).standard_normal((K, 100))
    bank = K * (n // 2) * 8
    # a budget below the bank: the plan is refused and nothing stays allocated
    free0 = torch.cuda.mem_get_info()[0]
    with pytest.raises(bfs.BfsError) as e:
        bfs.Plan(n, 4096.0, kappa=5.0, templates=temps, precision="f32", hbm_budget_bytes=bank // 2)
    assert e.value.status == bfs.BFS_ERR_OUT_OF_MEMORY
    # room for the bank and one small job, not for a job of 64 segments
    with bfs.Plan(n, 4096.0, kappa=5.0, templates=temps, precision="f32", tail_capacity=1024,
                  hbm_budget_bytes=bank + (4 << 20)) as plan:
        small = plan.job_bytes([n])
        big = plan.job_bytes([n] * 64)
        assert small < (4 << 20) < big
        ys = np.random.default_rng(32).standard_normal((64, n))
        with plan.filter(_dev(ys[0])) as job:
            job.fetch_tails()
        with pytest.raises(bfs.BfsError) as e:
            plan.filter(_dev(ys))
        assert e.value.status == bfs.BFS_ERR_OUT_OF_MEMORY
        with plan.filter(_dev(ys[1])) as job:  # the plan still works after the refusal
            assert job.fetch_sigma().shape == (1, K)
    torch.cuda.synchronize()
    assert abs(torch.cuda.mem_get_info()[0] - free0) < (64 << 20)


def test_segment_lengths_outside_the_plan_are_rejected(bfs):
    with bfs.Plan(1 << 14, 4096.0, kappa=5.0, templates=np.ones((2, 64)), precision="f32", n_min=1 << 12) as plan:
        y = torch.zeros(1 << 17, device="cuda")
        for lens in ([1 << 11], [1 << 15], [3000], [1 << 12, 1 << 16]):
            with pytest.raises(bfs.BfsError) as e:
                plan.filter(y, lengths=lens)
            assert e.value.status == bfs.BFS_ERR_INVALID_ARG, lens
        with pytest.raises(ValueError):  # extends past the buffer: caught by the binding
            plan.filter(y, lengths=[1 << 14], offsets=[(1 << 17) - 10])


def test_fp64_uneven_lengths_match_oracle(bfs):
    # FP64 plan over 2^11..2^14 (2^14 runs the split kernel in FP64) with segments of every length
    rng = np.random.default_rng(33)
    lens = [1 << 14, 1 << 11, 1 << 13, 1 << 12, 1 << 14]
    segs = [rng.standard_normal(n) for n in lens]
    temps = [rng.standard_normal(l) for l in (1, 100, 2048)]
    bank = np.zeros((3, 2048))
    for j, w in enumerate(temps):
        bank[j, :len(w)] = w
    kappa = 3.0
    with bfs.Plan(1 << 14, 4096.0, kappa=kappa, templates=bank, precision="f64", n_min=1 << 11) as plan:
        flat = torch.from_numpy(np.concatenate(segs)).cuda()
        with plan.filter(flat, lengths=lens) as job:
            tails, _ = job.fetch_tails()
            sig = job.fetch_sigma()
    out = oracle.search(segs, list(bank), kappa, keep_rho=True)
    assert np.max(np.abs(sig - out["sigma"]) / out["sigma"]) <= TOL["f64"]
    common, band = compare_tails(tails, out["tails"], out["sigma"], kappa, TOL["f64"],
                                 lambda s, j: out["rho"][s][j])
    assert common > 100 and band <= 2


def test_grid_of_2_to_32_work_items_matches_smaller_calls(bfs):
    # 8192 chirps x 512 segments of 2^16 samples = 8 * 1024 * 512 workgroups of 1024 threads,
    # 2^32 work items: more than one dispatch's 32-bit grid holds.  The library splits the
    # launch; the result equals eight calls of 64 segments, bitwise
    n, S = 1 << 16, 512
    ys = np.random.default_rng(34).standard_normal((S, n), dtype=np.float32)
    grid = bfs.Grid(128, 64, (350.0, 2000.0), (-500.0, 500.0), (1.0,))
    with bfs.Plan(n, 4096.0, kappa=5.5, grid=grid, precision="f32", tail_capacity=1 << 20) as plan:
        assert 8 * (plan.k // 8) * S * plan.threads_per_correlation == 1 << 32
        with plan.filter(_dev(ys)) as job:
            tails, total = job.fetch_tails()
            sig = job.fetch_sigma()
        parts_t, parts_s = [], []
        for s0 in range(0, S, 64):
            with plan.filter(_dev(ys[s0:s0 + 64])) as job:
                t, _ = job.fetch_tails()
                t["segment"] += s0
                parts_t.append(t)
                parts_s.append(job.fetch_sigma())
    assert total == len(tails) > 0
    assert np.array_equal(np.concatenate(parts_t), tails)
    assert np.array_equal(np.concatenate(parts_s), sig)


def test_device_sort_area_counts_pooled_buffers(bfs):
    # a released job's buffers stay allocated for reuse; the device sort area of a large
    # fetch must fit the budget with them counted, or they are given back first
    n, S, K = 4096, 3, 5
    rng = np.random.default_rng(35)
    ys = _dev(rng.standard_normal((S, n)).astype(np.float32))
    kw = dict(kappa=0.0, templates=rng.standard_normal((K, 300)), precision="f32", tail_capacity=S * K * n)

    def run(budget):
        with bfs.Plan(n, 4096.0, hbm_budget_bytes=budget, **kw) as plan:
            plan_b, job_b = plan.held_bytes(), plan.job_bytes([n] * S)
            j1 = plan.filter(ys)
            j2 = plan.filter(ys)
            j2.release()  # its buffer set goes to the pool
            tails, total = j1.fetch_tails()  # 61,440 tails: ordered on the device
            held = plan.held_bytes()
            j1.release()
        return tails, total, plan_b, job_b, held

    t0, tot0, plan_b, job_b, held0 = run(0)
    sort_b = held0 - plan_b - 2 * job_b
    assert tot0 == S * K * n and sort_b > job_b // 2
    budget = plan_b + job_b + sort_b + job_b // 2
    t1, tot1, _, _, held1 = run(budget)
    assert held1 <= budget
    assert held1 == plan_b + job_b + sort_b  # the pooled set was freed to make room
    assert tot1 == tot0 and np.array_equal(t0, t1)
