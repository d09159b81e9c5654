"""Benchmark of the matched-filter hot path on one MI355X.

A step is one pass of the hot path over one batch: the segment's forward real
FFT, the fused kernel over every template of the resident bank (product,
FP64 Parseval sigma, inverse FFT on chip, threshold, ballot compaction) and
the fetch of the sorted tails to the host.  The template bank (chirp
synthesis and forward FFT of every template) is built once per plan, as the
paper loads precomputed template transforms (Sec. 3.2, step (ii)); its build
time is reported beside the step rate.

Prints one JSON line.  With no flags: N = 1 GPU, workload C2 (N = 2^16,
8192 one-second chirps, kappa = 5, FP32), 400 timed steps after 50 warmups (the clocks settle during the warmups);
beside it the same with FP16-stored spectra, the batched form (C4: 64
segments of 2^14..2^17 samples against 65,536 chirps in one graph-replayed
job per step, autotuned kernels) and the serving form (C5: Poisson arrivals
of mixed-length segments against 262,144 FP16 chirp spectra, continuous
batching over several streams, p50/p99 latency).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12   # MI355X published FP32 vector peak, FLOP/s
PEAK_HBM = 8.0e12             # MI355X HBM3E, B/s

# HBM bytes per correlation-kernel launch on the C2 workload, from rocprofv3 FETCH_SIZE (x2,
# the factor a plain copy kernel of known size reads on this gfx950) + WRITE_SIZE (x1); valid
# only for the kernel sources and build flags they were taken on
# (profiles/corr_loop_kernel_C2_N65536_K8192_hbm.md).
MEASURED_TRAFFIC = {
    "b182d19ef50e545a": {"f32": 2.2069e+09, "f32-w16f": 1.0879e+09, "f32-w16b": 1.0888e+09, "f32 fused": 7.0090e+06},
}


def kernel_source_hash() -> str:
    import glob
    import hashlib

    h = hashlib.sha256()
    from paper_1708_01609_amd import build as b

    csrc = os.path.join(ROOT, "paper_1708_01609_amd", "csrc")
    # the correlation kernels' sources (their headers and the units that instantiate them;
    # not the host runtime, the tail sort or the runtime's small kernels) and the flags
    names = ["bfs_device.h", "bfs_fft3.h", "bfs_fused.h", "bfs_kernels.h", "bfs_kernelset.h", "bfs_records.h"]
    files = [os.path.join(csrc, n) for n in names] + glob.glob(os.path.join(csrc, "bfs_ks_*.hip"))
    for f in sorted(files):
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(b.FLAGS).replace(b.ROOT, "").encode())
    return h.hexdigest()[:16]


def nominal_flops(n: int) -> float:
    """5 N log2 N per correlation: the paper's FFT cost convention (Eq. 10, Sec. 3.2)."""
    return 5.0 * n * math.log2(n)


def algorithmic_flops(n: int) -> float:
    """Per correlation in the fused kernel: inverse real FFT (2.5 N log2 N), the complex
    product over N/2+1 bins (6 each) and the threshold (1 per lag)."""
    return 2.5 * n * math.log2(n) + 6.0 * (n // 2 + 1) + n


def fused_flops(n: int, length: float) -> float:
    """Per correlation with fused synthesis: the resident path's work plus the template's forward
    real FFT (2.5 N log2 N, its first radix-R pass pruned to the template's rows is not
    discounted), the unpack to the real spectrum (10 per bin) and the synthesis of L samples
    (the FP64 phase and taper are counted as 20 flops per sample)."""
    return algorithmic_flops(n) + 2.5 * n * math.log2(n) + 10.0 * (n // 2) + 20.0 * length


def algorithmic_bytes(n: int, spec_bytes: int) -> float:
    """Per correlation: one template spectrum row read from HBM (N/2 packed complex values)."""
    return (n // 2) * spec_bytes


def roof(flops: float, hbm_bytes: float, seconds: float) -> dict:
    """Achieved algorithmic FP32 VALU rate and HBM rate of `seconds` of kernel time, each as a
    fraction of the MI355X peak (157.3 TFLOP/s FP32 vector, 8 TB/s HBM)."""
    return {"achieved_tflops": flops / seconds / 1e12, "frac": flops / seconds / PEAK_FP32_VECTOR,
            "hbm_achieved_GBps": hbm_bytes / seconds / 1e9, "hbm_frac": hbm_bytes / seconds / PEAK_HBM}


SPEC_BYTES = {"f64": 16, "f32": 8, "f32-w16f": 4, "f32-w16b": 4}

# steps keep running after the requested warm-ups until this much wall time has passed, so
# the clocks reach their steady state whatever --warmup is
MIN_WARMUP_S = 1.5


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=400)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--workload", default="C2")
    p.add_argument("--precision", default="f32")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp16", action="store_true")
    p.add_argument("--cpu-templates", type=int, default=2048,
                   help="templates in the bounded oracle sample")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="also run a plain torch copy of this size (HBM counter calibration)")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-dense-bank", action="store_true")
    p.add_argument("--depth", type=int, default=2, help="filter calls in flight in the step loop")
    p.add_argument("--no-serving", action="store_true")
    p.add_argument("--batched-steps", type=int, default=5)
    p.add_argument("--serve-seconds", type=float, default=30.0,
                   help="simulated seconds of the C5 stream replayed at 1x for latency")
    p.add_argument("--serve-compressed-seconds", type=float, default=60.0,
                   help="simulated seconds of the C5 stream replayed as fast as arrivals allow")
    p.add_argument("--serve-speed", type=float, default=50.0)
    p.add_argument("--slots", type=int, default=4)
    p.add_argument("--max-batch", type=int, default=8)
    p.add_argument("--min-warmup-s", type=float, default=MIN_WARMUP_S,
                   help="warm-up wall time each timed plan runs at least (clock settling)")
    p.add_argument("--candidate", type=int, default=0,
                   help="force kernel candidate i > 0 of each length for the headline plan (0: autotuned)")
    p.add_argument("--fused", action="store_true",
                   help="the headline plan synthesises its templates per correlation (no resident bank)")
    p.add_argument("--only-headline", action="store_true",
                   help="time only the headline plan (and --no-fp16 aside, the 16-bit forms): for profilers")
    return p.parse_args()


def run_plan(bfs, torch, w, y_dev, precision, steps, warmup, depth=2, project=False, symmetric=False, kappa=None,
             kappa_hi=0.0, collect=None, pairs=False, fused=False, candidate=0):
    """Plan the workload, then time `steps` steps.  A step is one filter call (segment FFT +
    fused kernel over every template) and the fetch of its sorted tails; up to `depth` steps are
    queued on the stream, so the next step's kernels run while the host fetches and sorts the
    last one's tails (two concurrent streams measured slower: their kernels compete for the
    CUs).  Every timed step completes inside the timed region.  Warm-up runs the requested
    steps and then goes on until MIN_WARMUP_S has passed.  collect = (first, count): after
    timing, also return the dense rho and sigma of those templates and the last step's tails
    (for the comparison with the oracle, outside the timed region)."""
    from collections import deque

    import numpy as np

    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus, symmetric=symmetric)
    t0 = time.perf_counter()
    plan = bfs.Plan(w.n, w.fs, kappa=w.kappa if kappa is None else kappa, grid=grid, precision=precision,
                    tail_capacity=1 << 22, autotune=not candidate, project=project, kappa_hi=kappa_hi, pairs=pairs,
                    fused=fused, candidate=candidate)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    kernel = plan.kernel_info()
    corr_ms, job_ms, lat_ms, n_tails, last = [], [], [], 0, [None]

    def finish(item):
        nonlocal n_tails
        job, ts = item
        recs, total = job.fetch_projection() if project else job.fetch_tails()
        last[0] = recs
        lat_ms.append((time.perf_counter() - ts) * 1e3)
        c, t = job.timing()
        corr_ms.append(c)
        job_ms.append(t)
        n_tails = total
        job.release()

    def loop(n):
        q = deque()
        for i in range(n):
            q.append((plan.filter(y_dev), time.perf_counter()))
            if len(q) >= depth:
                finish(q.popleft())
        while q:
            finish(q.popleft())

    tw = time.perf_counter()
    loop(warmup)
    while time.perf_counter() - tw < MIN_WARMUP_S:
        loop(max(depth, 8))
    torch.cuda.synchronize()
    corr_ms.clear(), job_ms.clear(), lat_ms.clear()
    t0 = time.perf_counter()
    loop(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = {"bank_bytes": plan.bank_bytes, "threads": plan.threads_per_correlation,
            "job_device_ms": float(sum(job_ms) / len(job_ms)), "kernel": kernel}
    if collect is not None:
        first, count = collect
        rho, sig = [], []
        for j0 in range(first, first + count, 1024):
            c = min(1024, first + count - j0)
            r, sg = plan.correlate_dense(y_dev[:1], first=j0, count=c)
            rho.append(r[0].cpu().numpy())
            sig.append(sg[0].cpu().numpy())
        info["dense"] = {"first": first, "rho": np.concatenate(rho), "sigma": np.concatenate(sig),
                         "tails": last[0], "kappa": w.kappa if kappa is None else kappa}
    plan.close()
    return wall, build_s, corr_ms, lat_ms, n_tails, info


def library_c2r_context(torch, n, batch, kernel_rate, reps=10):
    """The platform FFT library's batched complex-to-real inverse transform of length n
    (torch.fft.irfft, which runs hipFFT / rocFFT on ROCm), timed with events over `reps`
    calls after three warm-up calls.  Context for the paper's efficiency figure, which states
    its whole correlation pipeline as about 65 % of clFFT's transform rate alone (Sec. 4);
    here the ratio is the correlation kernel's rate over the library's bare C2R rate at
    the same length and batch.  A measurement beside the product path, never part of it."""
    x = torch.randn(batch, n // 2 + 1, dtype=torch.complex64, device="cuda:0")
    out = torch.empty(batch, n, dtype=torch.float32, device="cuda:0")
    for _ in range(3):
        torch.fft.irfft(x, n=n, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.fft.irfft(x, n=n, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    rate = batch / (ms * 1e-3)
    del x, out
    torch.cuda.empty_cache()
    return {"library": "torch.fft.irfft (hipFFT / rocFFT), complex64 -> float32", "n": n, "batch": batch,
            "ms_per_batch": ms, "transforms_per_s": rate, "correlation_kernel_over_library_c2r": kernel_rate / rate}


def run_pairs(bfs, torch, w, args):
    """Detector pairs: the C2 segment (channel 0) and a second, independent channel of the same
    shape correlated as one pair (both channels through one complex inverse transform per
    template, Sec. 3.2 step (i)); a step is one filter call over the pair and its tail fetch."""
    import numpy as np
    from synthetic import make_segment

    ys = np.stack([make_segment(w, 0, channel=c)[0] for c in (0, 1)]).astype(np.float32)
    y_dev = torch.from_numpy(ys).cuda()
    wall, build_s, corr_ms, _, n_tails, info = run_plan(bfs, torch, w, y_dev, args.precision, args.steps,
                                                        args.warmup, args.depth, pairs=True)
    k = w.n_templates
    ks = float(np.mean(corr_ms)) * 1e-3
    corr = 2 * k  # real correlations per step
    return {"value": args.steps * corr / wall, "unit": "correlations/s", "kernel_rate": corr / ks,
            "roofline": roof(algorithmic_flops(w.n) * corr, algorithmic_bytes(w.n, SPEC_BYTES[args.precision]) * k,
                             ks),
            "ms_per_step": wall / args.steps * 1e3, "tails_per_step": n_tails, "kernel": info["kernel"]}


def run_batched(bfs, torch, steps, warmup):
    """C4: 64 segments of 2^14..2^17 samples, 65,536 chirps (tau 0.5/1/2 s), FP32, one filter call
    per step, captured once as a HIP graph and replayed, kernels autotuned at plan time; two
    steps in flight."""
    import numpy as np
    from synthetic import get_workload, make_segment

    w = get_workload("C4")
    segs = [make_segment(w, s)[0] for s in range(w.n_segments)]
    lens = [len(y) for y in segs]
    flat = torch.from_numpy(np.concatenate(segs).astype(np.float32)).cuda()
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    t0 = time.perf_counter()
    plan = bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision="f32", n_min=min(w.lengths),
                    graph=True, autotune=True)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    from collections import deque

    graph_ms, tails = [], 0

    def finish(job):
        nonlocal tails
        tails = job.fetch_tails()[1]
        graph_ms.append(job.timing()[0])
        job.release()

    def loop(n):
        # two steps in flight, as for C2: the host fetches and sorts one step's tails while
        # the next step's graph runs (each in-flight job holds its own buffers and graph)
        q = deque()
        for _ in range(n):
            q.append(plan.filter(flat, lengths=lens))
            if len(q) >= 2:
                finish(q.popleft())
        while q:
            finish(q.popleft())

    loop(max(warmup, 2))  # captures the graph of both buffer sets
    torch.cuda.synchronize()
    graph_ms.clear()
    t0 = time.perf_counter()
    loop(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k = w.n_templates
    corr = k * len(segs)
    flops = sum(algorithmic_flops(n) for n in lens) * k
    kernels = {str(n): plan.kernel_info(n) for n in sorted(set(lens))}
    # per length: the chosen kernel's time per correlation as the autotuner measured it at plan
    # build (HIP events around launches over 16 segments x 4096 templates in the chosen tile
    # order); the bank row is read once per tile of segments
    per_n = {}
    for n, ki in kernels.items():
        us = ki["tile_us"].get(ki["tile"], 0.0)
        if us > 0:
            per_n[n] = dict(roof(algorithmic_flops(int(n)), algorithmic_bytes(int(n), 8) / ki["tile"], us * 1e-6),
                            us_per_correlation=us, tile=ki["tile"])
    out = {"workload": f"C4: {w.description}", "value": steps * corr / wall, "unit": "correlations/s",
           "ms_per_step": wall / steps * 1e3, "graph_replay_ms": float(np.mean(graph_ms)),
           "correlations_per_step": corr, "segment_lengths": {str(n): lens.count(n) for n in sorted(set(lens))},
           "achieved_tflops_algorithmic": flops / (np.mean(graph_ms) * 1e-3) / 1e12,
           "frac_of_fp32_vector_peak": flops / (np.mean(graph_ms) * 1e-3) / PEAK_FP32_VECTOR,
           "roofline_per_n": per_n,
           "bank_bytes": plan.bank_bytes, "bank_build_and_tune_s": build_s, "tails_per_step": tails,
           "kernels": kernels}
    plan.close()
    return out


def run_dense_bank(bfs, torch, steps, warmup, precision="f32-w16f", collect=None, fused=False):
    """C3: the C2 segment against all 1,048,576 chirps (1024 f0 x 1024 fdot), kappa 5.5: 16-bit
    spectra resident (128 GiB), or FP32 with fused synthesis (each chirp made and transformed per
    correlation; a resident FP32 bank would take 256 GiB of the 288 GB)."""
    import numpy as np
    from synthetic import get_workload, make_segment

    w = get_workload("C3")
    y, _ = make_segment(w, 0)
    y_dev = torch.from_numpy(np.ascontiguousarray(y[None, :])).to(device="cuda:0", dtype=torch.float32)
    wall, build_s, corr_ms, lat_ms, n_tails, info = run_plan(bfs, torch, w, y_dev, precision, steps, warmup,
                                                             collect=collect, fused=fused)
    k = w.n_templates
    ks = float(np.mean(corr_ms)) * 1e-3
    flops = (fused_flops(w.n, w.taus[0] * w.fs) if fused else algorithmic_flops(w.n)) * k
    out = {"workload": f"C3: {w.description}", "precision": precision, "fused_synthesis": fused,
           "value": steps * k / wall, "unit": "correlations/s", "kernel_rate": k / ks,
           "roofline": roof(flops, 0.0 if fused else algorithmic_bytes(w.n, SPEC_BYTES[precision]) * k, ks),
           "ms_per_step": wall / steps * 1e3, "bank_bytes": info["bank_bytes"], "bank_build_s": build_s,
           "tails_per_step": n_tails}
    return out, info.get("dense")


def run_serving(bfs, torch, args):
    """C5: Poisson arrivals (8/s, 4 channels) of 2^14..2^17-sample segments against 262,144
    one-second chirps with FP16 spectra; continuous batching over several streams with HBM-budget
    admission.  A 1x replay gives the latency; a compressed replay the sustained rate under load."""
    from paper_1708_01609_amd.serve import GpuExecutor, Request, serve
    from synthetic import arrivals, get_workload, request_samples

    w = get_workload("C5")
    grid = bfs.Grid(w.n_f0, w.n_fdot, w.f0_range, w.fdot_range, w.taus)
    t0 = time.perf_counter()
    plan = bfs.Plan(w.n, w.fs, kappa=w.kappa, grid=grid, precision="f32-w16f", n_min=min(w.lengths),
                    autotune=True)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    horizon = max(args.serve_seconds, args.serve_compressed_seconds)
    arr = arrivals(w, horizon)
    reqs = [Request(a.index, a.time, request_samples(w, a)[0], a.channel) for a in arr]
    ex = GpuExecutor(plan, slots=args.slots, max_batch=args.max_batch)
    budget = args.slots * plan.job_bytes([w.n] * args.max_batch)
    # warm the executor's streams and the job-buffer pool
    serve(ex, reqs[: 2 * args.max_batch], slots=args.slots, max_batch=args.max_batch, budget_bytes=budget,
          speed=1e6)
    def report(done, total, wall):
        print(f"serving: {done}/{total} requests after {wall:.0f} s", file=sys.stderr, flush=True)

    rt = serve(ex, [r for r in reqs if r.arrival < args.serve_seconds], slots=args.slots,
               max_batch=args.max_batch, budget_bytes=budget, speed=1.0, progress=report)
    sat = serve(ex, [r for r in reqs if r.arrival < args.serve_compressed_seconds], slots=args.slots,
                max_batch=args.max_batch, budget_bytes=budget, speed=args.serve_speed, progress=report)
    k = w.n_templates
    sat_sum = sat.summary(k)
    sat_reqs = [r for r in reqs if r.arrival < args.serve_compressed_seconds and r.rid in sat.results]
    flops = sum(algorithmic_flops(len(r.samples)) for r in sat_reqs) * k
    hbm = sum(algorithmic_bytes(len(r.samples), 4) for r in sat_reqs) * k
    sat_sum["roofline_wall_clock"] = roof(flops, hbm, sat.wall_s) if sat.wall_s > 0 else None
    out = {"workload": f"C5: {w.description}", "bank_bytes": plan.bank_bytes, "bank_build_and_tune_s": build_s,
           "slots": args.slots, "max_batch": args.max_batch, "hbm_budget_bytes_jobs": budget,
           "realtime": dict(rt.summary(k), simulated_s=args.serve_seconds, speed=1.0),
           "compressed": dict(sat_sum, simulated_s=args.serve_compressed_seconds, speed=args.serve_speed)}
    plan.close()
    return out


# Tolerance on |rho_gpu - rho_oracle| / sigma_oracle per precision form (the stated targets: FP32
# path 1e-4 sigma, reduced-storage path 2e-3 sigma).  A template whose sigma lies below
# RELAX * ||w|| rms(y) sits almost wholly outside the data band; FP32 rounding follows that input
# scale, so there the scale of the bound is RELAX * ||w|| rms(y) instead of sigma.
ERR_TOL = {"f64": 1e-9, "f32": 1e-4, "f32-w16f": 2e-3, "f32-w16b": 2e-3}
RELAX = 0.1


def error_vs_oracle(w, y, dense, precision, block=512):
    """Compare one precision form's dense rho, sigma and filter-path tails (segment 0, templates
    dense['first'] ..) with the FP64 oracle: the largest |rho error| / sigma and |sigma error| / sigma
    over the templates held to the bound strictly, the relaxed ones apart, and the tail sets
    (equal outside a +-tol band around kappa sigma).  Checker leg: runs the oracle, never timed."""
    import numpy as np

    import oracle

    f0, fd, tau = w.template_params()
    first, rho_g, sig_g = dense["first"], dense["rho"], dense["sigma"]
    kappa, tails = dense["kappa"], dense["tails"]
    count = len(sig_g)
    tol = ERR_TOL[precision]
    y64 = np.asarray(y, dtype=np.float64)
    rms_y = float(np.sqrt(np.mean(y64 * y64)))
    t0 = tails[tails["segment"] == 0]
    t0 = t0[(t0["template"] >= first) & (t0["template"] < first + count)]
    err, s_o, floor = np.empty(count), np.empty(count), np.empty(count)
    n_or = n_common = n_band = n_out = 0
    for b0 in range(0, count, block):
        ids = list(range(first + b0, first + min(count, b0 + block)))
        bank = oracle.template_bank(f0, fd, tau, w.fs, ids=ids)
        rho_o = oracle.correlate_fft(y64, np.array(bank))
        so = oracle.sigma_time(rho_o)
        sl = slice(b0, b0 + len(ids))
        err[sl] = np.max(np.abs(rho_g[sl].astype(np.float64) - rho_o), axis=1)
        s_o[sl] = so
        floor[sl] = [float(np.sqrt(np.dot(t, t))) * rms_y for t in bank]
        lo = np.searchsorted(t0["template"], ids[0], side="left")
        for r, j in enumerate(ids):
            hi = np.searchsorted(t0["template"], j, side="right")
            lags_g = set(int(v) for v in t0["lag"][lo:hi])
            lo = hi
            lags_o = set(int(v) for v in oracle.threshold_tails(rho_o[r], so[r], kappa))
            n_or += len(lags_o)
            n_common += len(lags_o & lags_g)
            scale = max(so[r], RELAX * floor[b0 + r])
            for lag in lags_o ^ lags_g:
                if abs(abs(rho_o[r, lag]) - kappa * so[r]) <= tol * scale:
                    n_band += 1
                else:
                    n_out += 1
        del rho_o
    rel = s_o < RELAX * floor
    sig_err = np.abs(sig_g - s_o)
    scale = np.maximum(s_o, RELAX * floor)
    out = {"templates": f"{first}..{first + count - 1}", "precision": precision, "tol_sigma": tol,
           "max_rho_err_over_sigma": float(np.max(err[~rel] / s_o[~rel])),
           "max_sigma_err_over_sigma": float(np.max(sig_err[~rel] / s_o[~rel])),
           "n_relaxed": int(rel.sum()),
           "relaxed_max_rho_err_over_scale": float(np.max(err[rel] / scale[rel])) if rel.any() else None,
           "tails_oracle": n_or, "tails_gpu": int(len(t0)), "tails_common": n_common,
           "tails_differ_in_band": n_band, "tails_differ_outside_band": n_out}
    out["meets_tol"] = bool(np.all(err <= tol * scale) and np.all(sig_err <= tol * scale) and n_out == 0)
    return out


def cpu_baseline(w, y, n_templates, min_seconds=10.0, max_passes=32):
    """The oracle as it stands on this host's cores: template synthesis, FFT correlation and
    threshold of segment 0 against blocks of n_templates templates, the blocks cycling over
    the whole bank, until at least min_seconds have passed (at most max_passes blocks)."""
    import oracle

    f0, fd, tau = w.template_params()
    blk = min(n_templates, w.n_templates)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    passes, dt, done = 0, 0.0, 0
    while passes < max_passes and (passes == 0 or dt < min_seconds):
        first = (passes * blk) % w.n_templates
        ids = list(range(first, min(first + blk, w.n_templates)))
        t0 = time.perf_counter()
        bank = oracle.template_bank(f0, fd, tau, w.fs, ids=ids)
        oracle.search([y.astype("float64")], bank, w.kappa)
        dt += time.perf_counter() - t0
        done += len(ids)
        passes += 1
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": done / dt, "unit": "correlations/s", "cores": cores, "kind": "oracle",
            "sample": f"{w.name}: segment 0 against {done} templates in blocks of {blk} cycling over the "
                      f"{w.n_templates} (FP64 scipy.fft, template synthesis included), {dt:.1f} s", "cpu": cpu}


def main():
    global MIN_WARMUP_S
    args = parse()
    MIN_WARMUP_S = args.min_warmup_s
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; multi-GPU runs are not supported "
              "(it would shard by templates or segments, one resident bank slice per GPU, with no "
              "exchange between GPUs)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1708_01609_amd import build as b

    if not os.path.exists(b.LIB):
        b.build()
    from paper_1708_01609_amd import bfsearch as bfs
    from synthetic import get_workload, make_segment

    w = get_workload(args.workload)
    y, _ = make_segment(w, 0)
    dt = torch.float64 if args.precision == "f64" else torch.float32
    y_dev = torch.from_numpy(np.ascontiguousarray(y[None, :])).to(device="cuda:0", dtype=dt)

    check = not args.no_cpu_baseline and w.name == "C2"  # the checker leg compares with the oracle
    dense = {}  # precision form -> (workload, segment, GPU outputs) for the checker leg
    wall, build_s, corr_ms, lat_ms, n_tails, info = run_plan(
        bfs, torch, w, y_dev, args.precision, args.steps, args.warmup, args.depth,
        collect=(0, w.n_templates) if check else None, fused=args.fused, candidate=args.candidate)
    if check:
        dense[f"{w.name} {args.precision}{' fused' if args.fused else ''}"] = (w, y, info.pop("dense"), args.precision)
    k = w.n_templates
    value = args.steps * k / wall
    corr_avg_s = float(np.mean(corr_ms)) * 1e-3
    spec_bytes = SPEC_BYTES[args.precision]
    flops_corr = fused_flops(w.n, w.taus[0] * w.fs) if args.fused else algorithmic_flops(w.n)
    r = roof(flops_corr * k, 0.0 if args.fused else algorithmic_bytes(w.n, spec_bytes) * k, corr_avg_s)
    line = {
        "metric": "correlations/s (N=2^16, tau=1 s) on 1 MI355X",
        "value": value,
        "unit": "correlations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.description}", "n": w.n, "templates": k, "segments": 1,
                   "kappa": w.kappa, "precision": args.precision, "fused_synthesis": args.fused},
        "roofline": {
            "bound": "alu",
            "kernel": ("corr_fused_kernel (synthesis, forward FFT, product, sigma, inverse FFT, threshold)"
                       if args.fused else
                       ("corr_loop_kernel" if info["kernel"].get("loop") else "corr_kernel")
                       + " (fused product, sigma, inverse FFT, threshold, compaction)"),
            "achieved": r["achieved_tflops"],
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": r["frac"],
            "traffic": MEASURED_TRAFFIC.get(kernel_source_hash(), {}).get(
                args.precision + (" fused" if args.fused else "")) if w.name == "C2" else None,
            "flops_per_correlation": flops_corr,
            "correlations_per_launch": k,
            "kernel_ms_avg": corr_avg_s * 1e3,
            "hbm_algorithmic_GBps": r["hbm_achieved_GBps"],
            "hbm_frac": r["hbm_frac"],
            "hbm_peak_GBps": PEAK_HBM / 1e9,
        },
        "kernel_rate": k / corr_avg_s,
        "nominal_tflops": nominal_flops(w.n) * value / 1e12,
        "pipeline_depth": args.depth,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(np.max(lat_ms))},
        "job_device_ms": info["job_device_ms"],
        "kernel": info["kernel"],
        "bank_build_and_tune_s": build_s,
        "bank_bytes": info["bank_bytes"],
        "tails_per_step": n_tails,
    }
    if not args.no_fp16 and args.precision == "f32":
        # reduced-storage form: template spectra stored FP16 / BF16, FFT and accumulation FP32
        for prec, key in (("f32-w16f", "fp16_spectra"), ("f32-w16b", "bf16_spectra")):
            wall16, build16, corr16, _, _, info16 = run_plan(bfs, torch, w, y_dev, prec, args.steps, args.warmup,
                                                             args.depth, collect=(0, k) if check else None)
            ks16 = float(np.mean(corr16)) * 1e-3
            line[key] = {"value": args.steps * k / wall16, "kernel_rate": k / ks16,
                         "roofline": roof(algorithmic_flops(w.n) * k, algorithmic_bytes(w.n, 4) * k, ks16),
                         "traffic": MEASURED_TRAFFIC.get(kernel_source_hash(), {}).get(prec),
                         "ms_per_step": wall16 / args.steps * 1e3, "bank_build_s": build16,
                         "bank_bytes": info16["bank_bytes"]}
            if check:
                dense[f"{w.name} {prec}"] = (w, y, info16.pop("dense"), prec)
    if args.copy_calibration_mib:
        # plain kernels of known traffic for scaling the HBM counters: fill writes X bytes,
        # neg reads X and writes X, sum reads X
        nbytes = args.copy_calibration_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        c = torch.empty_like(a)
        torch.neg(a, out=c)
        _ = float(a.sum())
        torch.cuda.synchronize()
        line["calibration_bytes"] = nbytes
    forms = args.workload == "C2" and not args.only_headline
    if forms:
        # the paper's default output: per-lag max projection over templates (Sec. 3.3)
        wallp, _, corrp, _, n_peaks, _ = run_plan(bfs, torch, w, y_dev, args.precision, args.steps, args.warmup,
                                                 args.depth, project=True)
        line["max_projection"] = {"value": args.steps * k / wallp, "kernel_rate": k / (np.mean(corrp) * 1e-3),
                                  "ms_per_step": wallp / args.steps * 1e3, "lags_per_step": n_peaks}
        # time-symmetric bank (chirp plus its reversal) and a finite tail band 3 sigma < |rho| < 3.5 sigma
        walls, builds, corrs, _, n_sym, _ = run_plan(bfs, torch, w, y_dev, args.precision, args.steps, args.warmup,
                                                    args.depth, symmetric=True)
        line["symmetric_bank"] = {"value": args.steps * k / walls, "kernel_rate": k / (np.mean(corrs) * 1e-3),
                                  "bank_build_and_tune_s": builds, "tails_per_step": n_sym}
        wallb, _, corrb, _, n_band, _ = run_plan(bfs, torch, w, y_dev, args.precision, args.steps, args.warmup,
                                                args.depth, kappa=3.0, kappa_hi=3.5)
        line["band_threshold"] = {"kappa": 3.0, "kappa_hi": 3.5, "value": args.steps * k / wallb,
                                  "kernel_rate": k / (np.mean(corrb) * 1e-3), "tails_per_step": n_band}
        line["detector_pairs"] = run_pairs(bfs, torch, w, args)
        line["library_c2r_context"] = library_c2r_context(torch, w.n, k, k / corr_avg_s)
    if forms and args.precision == "f32":
        # fused synthesis on the C2 workload: the same search with no resident bank
        wallf, buildf, corrf, _, _, infof = run_plan(bfs, torch, w, y_dev, "f32", args.steps, args.warmup,
                                                     args.depth, collect=(0, k) if check else None, fused=True)
        ksf = float(np.mean(corrf)) * 1e-3
        line["fused_synthesis"] = {"value": args.steps * k / wallf, "kernel_rate": k / ksf,
                                   "roofline": roof(fused_flops(w.n, w.taus[0] * w.fs) * k, 0.0, ksf),
                                   "traffic": MEASURED_TRAFFIC.get(kernel_source_hash(), {}).get("f32 fused"),
                                   "ms_per_step": wallf / args.steps * 1e3, "plan_build_s": buildf,
                                   "bank_bytes": infof["bank_bytes"], "kernel": infof["kernel"]}
        if check:
            dense[f"{w.name} f32 fused"] = (w, y, infof.pop("dense"), "f32")
    if not args.no_dense_bank and forms:
        for prec, key, fused in (("f32-w16f", "dense_bank_fp16", False), ("f32-w16b", "dense_bank_bf16", False),
                                 ("f32", "dense_bank_fp32_fused", True)):
            out, d3 = run_dense_bank(bfs, torch, 3, 1, precision=prec, collect=(0, 4096) if check else None,
                                     fused=fused)
            line[key] = out
            if check:
                dense[f"C3 {prec}{' fused' if fused else ''}"] = (get_workload("C3"),
                                                                  make_segment(get_workload("C3"), 0)[0], d3, prec)
    if not args.no_batched and forms:
        line["batched"] = run_batched(bfs, torch, args.batched_steps, 1)
    if not args.no_serving and forms:
        line["serving"] = run_serving(bfs, torch, args)
    if not args.no_cpu_baseline:
        # checker leg: the oracle timed on the host cores, and every precision form's error
        # against it (outside every timed region)
        line["cpu_baseline"] = cpu_baseline(w, y, args.cpu_templates)
        if dense:
            line["error_vs_oracle"] = {name: error_vs_oracle(wd, yd, dd, prec)
                                       for name, (wd, yd, dd, prec) in dense.items()}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
