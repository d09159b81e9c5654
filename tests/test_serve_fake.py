"""Scheduler of the serving form, driven on the CPU by a stand-in executor.

The stand-in computes each request's result with the FP64 oracle and
completes a job after a service time proportional to its correlations on a
virtual clock, so admission, slot and budget limits, batching and result
routing are checked without a GPU.
"""
import numpy as np
import pytest

import oracle
from paper_1708_01609_amd.serve import Request, serve


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    def __init__(self, bank, kappa, clock, us_per_sample=0.05, fixed_bytes=1000):
        self.bank, self.kappa, self.clock = bank, kappa, clock
        self.us_per_sample = us_per_sample
        self.fixed_bytes = fixed_bytes
        self.log = []          # (event, time, slot, rids)
        self.busy = {}

    def job_bytes(self, lengths):
        return self.fixed_bytes + sum(4 * n for n in lengths) + 8 * len(lengths) * len(self.bank)

    def submit(self, slot, reqs):
        assert slot not in self.busy, "slot reused while its job is in flight"
        self.busy[slot] = True
        t = self.clock.now()
        service = 1e-6 * self.us_per_sample * sum(len(r.samples) for r in reqs) * len(self.bank)
        self.log.append(("submit", t, slot, [r.rid for r in reqs]))
        out = oracle.search([r.samples for r in reqs], self.bank, self.kappa)
        return {"slot": slot, "ready_at": t + service, "out": out, "n": len(reqs)}

    def ready(self, h):
        return self.clock.now() >= h["ready_at"]

    def collect(self, h):
        del self.busy[h["slot"]]
        self.log.append(("done", self.clock.now(), h["slot"], None))
        out = h["out"]
        t = out["tails"]
        return [(t[t["segment"] == s], out["sigma"][s], True) for s in range(h["n"])]


class OverflowingExecutor(FakeExecutor):
    """Keeps at most `cap` tails per job, like the device buffer, and says so."""

    def __init__(self, *a, cap=5, **kw):
        super().__init__(*a, **kw)
        self.cap = cap

    def collect(self, h):
        per = super().collect(h)
        total = sum(len(t) for t, _, _ in per)
        if total <= self.cap:
            return per
        kept, out = 0, []
        for t, sg, _ in per:
            k = max(0, min(len(t), self.cap - kept))
            kept += k
            out.append((t[:k], sg, False))
        return out


class FailingExecutor(FakeExecutor):
    """Raises in submit for jobs holding a request id in fail_submit, in collect for fail_collect."""

    def __init__(self, *a, fail_submit=(), fail_collect=(), **kw):
        super().__init__(*a, **kw)
        self.fail_submit, self.fail_collect = set(fail_submit), set(fail_collect)

    def submit(self, slot, reqs):
        if self.fail_submit & {r.rid for r in reqs}:
            raise RuntimeError("submit failed")
        h = super().submit(slot, reqs)
        h["rids"] = {r.rid for r in reqs}
        return h

    def collect(self, h):
        if self.fail_collect & h["rids"]:
            del self.busy[h["slot"]]
            raise RuntimeError("collect failed")
        return super().collect(h)


def _requests(count, rate, seed, lengths=(256, 512, 1024)):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    return [Request(i, float(t[i]), rng.standard_normal(int(rng.choice(lengths)))) for i in range(count)]


@pytest.fixture
def bank():
    rng = np.random.default_rng(5)
    return [rng.standard_normal(64) for _ in range(6)]


def test_every_request_is_served_once_with_its_own_result(bank):
    clk = VirtualClock()
    ex = FakeExecutor(bank, 3.0, clk)
    reqs = _requests(40, rate=200.0, seed=1)
    st = serve(ex, reqs, slots=3, max_batch=4, clock=clk.now, sleep=clk.sleep)
    assert sorted(st.results) == list(range(40)) and not st.rejected
    for r in reqs:
        alone = oracle.search([r.samples], bank, 3.0)
        got = st.results[r.rid]
        assert np.array_equal(got.sigma, alone["sigma"][0])
        assert np.array_equal(got.tails["template"], alone["tails"]["template"])
        assert np.array_equal(got.tails["lag"], alone["tails"]["lag"])
        assert np.all(got.tails["segment"] == r.rid)
        assert got.latency >= 0 and got.queue_wait >= 0
    assert st.max_inflight <= 3
    assert all(len(e[3]) <= 4 for e in ex.log if e[0] == "submit")


def test_admission_is_fifo_and_overlaps_jobs(bank):
    # arrivals faster than service: jobs overlap (several in flight), batches grow, order kept
    clk = VirtualClock()
    ex = FakeExecutor(bank, 3.0, clk, us_per_sample=0.5)
    reqs = _requests(30, rate=2000.0, seed=2)
    st = serve(ex, reqs, slots=2, max_batch=8, clock=clk.now, sleep=clk.sleep)
    order = [rid for e in ex.log if e[0] == "submit" for rid in e[3]]
    assert order == sorted(order) == list(range(30))
    assert st.max_inflight == 2
    assert max(len(e[3]) for e in ex.log if e[0] == "submit") > 1
    # continuous batching: a job is admitted while another is still in flight
    inflight, overlapped = 0, False
    for e in ex.log:
        inflight += 1 if e[0] == "submit" else -1
        overlapped |= inflight > 1
    assert overlapped


def test_hbm_budget_limits_inflight_bytes_and_rejects_oversize(bank):
    clk = VirtualClock()
    ex = FakeExecutor(bank, 3.0, clk, us_per_sample=0.5)
    reqs = _requests(20, rate=5000.0, seed=3)
    one = max(ex.job_bytes([len(r.samples)]) for r in reqs)
    budget = 2 * one + 10
    st = serve(ex, reqs, slots=4, max_batch=8, budget_bytes=budget, clock=clk.now, sleep=clk.sleep)
    assert st.max_inflight_bytes <= budget and not st.rejected and len(st.results) == 20
    # a request whose job alone exceeds the budget is rejected, the rest are served
    big = Request(99, 0.0, np.zeros(1 << 14))
    st = serve(ex, reqs + [big], slots=4, max_batch=8, budget_bytes=budget, clock=clk.now, sleep=clk.sleep)
    assert st.rejected == [99] and len(st.results) == 20


def test_replay_speed_scales_arrivals(bank):
    clk = VirtualClock()
    ex = FakeExecutor(bank, 3.0, clk, us_per_sample=1e-4)
    reqs = _requests(10, rate=10.0, seed=4)
    st = serve(ex, reqs, slots=2, max_batch=2, speed=10.0, clock=clk.now, sleep=clk.sleep)
    last = max(r.arrival for r in reqs)
    assert st.wall_s >= last / 10.0 and st.wall_s < last / 10.0 + 0.05
    s = st.summary(len(bank))
    assert s["requests"] == 10 and s["correlations"] == 60 and s["latency_ms"]["p99"] >= s["latency_ms"]["p50"]


def test_invalid_parameters():
    with pytest.raises(ValueError):
        serve(None, [], slots=0)


def test_overflowed_jobs_flag_their_requests_incomplete(bank):
    # a job whose tails overflow returns partial lists: every request of that job is flagged,
    # counted as truncated, and the complete ones keep their full result
    clk = VirtualClock()
    ex = OverflowingExecutor(bank, 1.0, clk, cap=40)
    reqs = _requests(12, rate=100.0, seed=6)
    st = serve(ex, reqs, slots=2, max_batch=3, clock=clk.now, sleep=clk.sleep)
    assert sorted(st.results) == list(range(12))
    flagged = {rid for rid, r in st.results.items() if not r.complete}
    assert flagged and st.summary(len(bank))["truncated"] == len(flagged)
    for rid, r in st.results.items():
        alone = oracle.search([reqs[rid].samples], bank, 1.0)
        if r.complete:
            assert len(r.tails) == len(alone["tails"])
        else:
            assert len(r.tails) <= len(alone["tails"])
    # jobs are flagged as a whole: requests sharing a job share the flag
    by_job = {}
    for r in st.results.values():
        by_job.setdefault(r.job, set()).add(r.complete)
    assert all(len(v) == 1 for v in by_job.values())


def test_executor_errors_fail_only_their_job(bank):
    # submit raising for request 3's job, collect raising for request 7's: those jobs' requests
    # fail, their slots come back, and every other request is served with its own result
    clk = VirtualClock()
    ex = FailingExecutor(bank, 3.0, clk, fail_submit={3}, fail_collect={7})
    reqs = _requests(16, rate=50.0, seed=7)
    st = serve(ex, reqs, slots=2, max_batch=2, clock=clk.now, sleep=clk.sleep)
    failed = {rid for rid, _ in st.failed}
    assert 3 in failed and 7 in failed
    assert failed.isdisjoint(st.results) and len(failed) + len(st.results) == 16
    assert len(failed) <= 4 and not ex.busy
    s = st.summary(len(bank))
    assert s["failed"] == len(failed) and s["requests"] == len(st.results)
    for rid, r in st.results.items():
        alone = oracle.search([reqs[rid].samples], bank, 3.0)
        assert np.array_equal(r.sigma, alone["sigma"][0])
