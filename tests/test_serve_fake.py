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
        return [(t[t["segment"] == s], out["sigma"][s]) for s in range(h["n"])]


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
