"""Serving form: continuous batching of arriving segment requests.

Requests (one strain segment each, any length the plan accepts) arrive over
time.  The scheduler keeps up to `slots` jobs in flight, one per HIP stream,
so their kernels overlap on the device.  Whenever a slot is free it admits
the requests that are waiting, oldest first, as one job of up to `max_batch`
segments of mixed lengths, as long as the job's device bytes fit the HBM
budget next to the jobs already in flight.  A completion poller collects each
finished job, splits its tails per request and records the request's latency
from arrival to results on the host.

The scheduler is host logic only and talks to an executor:
    job_bytes(lengths) -> int            device bytes of a job of these lengths
    submit(slot, requests) -> handle     queue a job on the slot's stream
    ready(handle) -> bool                non-blocking completion check
    collect(handle) -> [(tails, sigma, complete)]
                                         per request: its tails (segment field
                                         = position in the job), sigma [K] and
                                         whether the tail list is complete
GpuExecutor runs jobs through the library; tests drive the scheduler with a
CPU stand-in.  Each correlation is computed by one workgroup with a fixed
reduction order, so a request's result does not depend on which requests
share its job.  A job whose tails overflowed the device buffer returns its
requests flagged incomplete (the device counts every tail but keeps only as
many as fit, in no particular order), and they are counted as truncated.  An
executor error in submit or collect fails that job's requests only; the slot
is freed and serving goes on.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds since the start of the stream
    samples: np.ndarray     # host samples (float32 for FP32 plans, float64 for FP64)
    channel: int = 0


@dataclass
class Result:
    rid: int
    tails: np.ndarray       # tail records of this request (segment field = rid)
    sigma: np.ndarray       # [K]
    arrival_wall: float
    admit_wall: float
    done_wall: float
    job: int                # sequence number of the job it ran in
    batch: int              # requests in that job
    complete: bool = True   # False: the job's tails overflowed, this list may miss some

    @property
    def latency(self) -> float:
        return self.done_wall - self.arrival_wall

    @property
    def queue_wait(self) -> float:
        return self.admit_wall - self.arrival_wall


@dataclass
class ServeStats:
    results: dict = field(default_factory=dict)
    rejected: list = field(default_factory=list)
    failed: list = field(default_factory=list)    # (rid, error text) of requests whose job raised
    wall_s: float = 0.0
    jobs: int = 0
    max_inflight: int = 0
    max_inflight_bytes: int = 0

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.results.values()])

    def summary(self, k_templates: int) -> dict:
        lat = self.latencies() * 1e3
        n = len(self.results)
        return {
            "requests": n,
            "rejected": len(self.rejected),
            "failed": len(self.failed),
            "truncated": sum(1 for r in self.results.values() if not r.complete),
            "jobs": self.jobs,
            "mean_batch": n / max(self.jobs, 1),
            "max_inflight_jobs": self.max_inflight,
            "max_inflight_bytes": self.max_inflight_bytes,
            "wall_s": self.wall_s,
            "correlations": n * k_templates,
            "correlations_per_s": n * k_templates / self.wall_s if self.wall_s > 0 else 0.0,
            "latency_ms": {
                "p50": float(np.percentile(lat, 50)) if n else None,
                "p99": float(np.percentile(lat, 99)) if n else None,
                "max": float(np.max(lat)) if n else None,
            },
        }


def serve(executor, requests, slots: int = 4, max_batch: int = 16, budget_bytes: int = 0,
          speed: float = 1.0, poll_s: float = 2e-4, clock=time.perf_counter, sleep=time.sleep,
          progress=None, progress_every_s: float = 30.0) -> ServeStats:
    """Replay `requests` (arrival times in stream seconds) at `speed` x real time and serve them.

    budget_bytes: device bytes the in-flight jobs may hold together (0: no limit beyond the
    executor's own).  A request whose job alone exceeds the budget is rejected.  Returns
    per-request results and totals; latencies are wall-clock seconds from the request's
    (scaled) arrival to its results on the host.  progress(done, total, wall_s), if given,
    is called about every progress_every_s seconds."""
    if slots < 1 or max_batch < 1 or speed <= 0:
        raise ValueError("slots, max_batch and speed must be positive")
    stats = ServeStats()
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    waiting: deque = deque()
    free = list(range(slots))[::-1]
    inflight: dict = {}     # slot -> (handle, requests, bytes, admit_wall, job id)
    inflight_bytes = 0
    t0 = clock()
    next_report = t0 + progress_every_s
    n_total = len(pending)

    def arrival_wall(r):
        return t0 + r.arrival / speed

    while pending or waiting or inflight:
        now = clock()
        if progress is not None and now >= next_report:
            progress(len(stats.results) + len(stats.rejected) + len(stats.failed), n_total, now - t0)
            next_report = now + progress_every_s
        while pending and arrival_wall(pending[0]) <= now:
            waiting.append(pending.popleft())
        progressed = False
        # completions
        for slot in list(inflight):
            handle, reqs, nbytes, t_adm, jid = inflight[slot]
            try:
                if not executor.ready(handle):
                    continue
                per_req = executor.collect(handle)
            except Exception as e:  # the job failed: its requests only
                stats.failed.extend((r.rid, repr(e)) for r in reqs)
                per_req = None
            t_done = clock()
            for r, res in zip(reqs, per_req or ()):
                tails, sigma = res[0], res[1]
                complete = bool(res[2]) if len(res) > 2 else True
                t = tails.copy()
                if len(t):
                    t["segment"] = r.rid
                stats.results[r.rid] = Result(r.rid, t, sigma, arrival_wall(r), t_adm, t_done, jid, len(reqs),
                                              complete)
            inflight_bytes -= nbytes
            del inflight[slot]
            free.append(slot)
            progressed = True
        # admission: one job per free slot, oldest waiting requests first
        while free and waiting:
            batch, lens, nbytes = [], [], 0
            while waiting and len(batch) < max_batch:
                cand = lens + [len(waiting[0].samples)]
                b = executor.job_bytes(cand)
                if budget_bytes and inflight_bytes + b > budget_bytes:
                    break
                batch.append(waiting.popleft())
                lens, nbytes = cand, b
            if not batch:
                if not inflight:  # the oldest request alone does not fit an empty device
                    stats.rejected.append(waiting.popleft().rid)
                    continue
                break
            slot = free.pop()
            t_adm = clock()
            try:
                handle = executor.submit(slot, batch)
            except Exception as e:  # nothing was queued: fail these requests, keep the slot
                stats.failed.extend((r.rid, repr(e)) for r in batch)
                free.append(slot)
                progressed = True
                continue
            inflight[slot] = (handle, batch, nbytes, t_adm, stats.jobs)
            stats.jobs += 1
            inflight_bytes += nbytes
            stats.max_inflight = max(stats.max_inflight, len(inflight))
            stats.max_inflight_bytes = max(stats.max_inflight_bytes, inflight_bytes)
            progressed = True
        if not progressed:
            if inflight:
                sleep(poll_s)
            elif pending:
                sleep(max(0.0, min(arrival_wall(pending[0]) - clock(), 0.05)))
    stats.wall_s = clock() - t0
    return stats


class GpuExecutor:
    """Runs serving jobs through the library: one torch stream (default priority) per slot,
    pinned host staging and a device buffer per slot, reused job after job."""

    def __init__(self, plan, slots: int, max_batch: int, device: str = "cuda:0"):
        import torch

        self.torch = torch
        self.plan = plan
        dt = torch.float64 if plan.sample_dtype == "float64" else torch.float32
        cap = max_batch * plan.n
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.host = [torch.empty(cap, dtype=dt).pin_memory() for _ in range(slots)]
        self.dev = [torch.empty(cap, dtype=dt, device=device) for _ in range(slots)]

    def job_bytes(self, lengths) -> int:
        return self.plan.job_bytes(lengths)

    def submit(self, slot, reqs):
        torch = self.torch
        lens = [len(r.samples) for r in reqs]
        total = sum(lens)
        host = self.host[slot][:total].numpy()
        o = 0
        for r in reqs:
            host[o:o + len(r.samples)] = r.samples
            o += len(r.samples)
        st = self.streams[slot]
        with torch.cuda.stream(st):
            self.dev[slot][:total].copy_(self.host[slot][:total], non_blocking=True)
        job = self.plan.filter(self.dev[slot][:total], lengths=lens, stream=st)
        return job

    def ready(self, job) -> bool:
        return job.done()

    def collect(self, job):
        try:
            tails, total = job.fetch_tails(allow_overflow=True)
            sigma = job.fetch_sigma()
        finally:
            job.release()
        # on overflow the device kept an arbitrary subset: no request's list is known complete
        complete = total == len(tails)
        seg = tails["segment"]
        return [(tails[seg == s], sigma[s], complete) for s in range(job.n_segments)]
