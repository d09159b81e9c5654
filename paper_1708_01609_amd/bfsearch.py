"""ctypes binding of libbfsearch.so (include/bfsearch.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind the C ABI.  torch supplies device memory (the segment tensor,
diagnostic outputs) and the stream handle.  If the library is not built this
module raises at import; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfsearch.so")

BFS_OK = 0
BFS_ERR_INVALID_ARG = -1
BFS_ERR_OUT_OF_MEMORY = -2
BFS_ERR_HIP = -3
BFS_ERR_TAIL_OVERFLOW = -4
BFS_ERR_UNSUPPORTED = -5
BFS_ERR_SCRATCH_LIMIT = -6
NOALLOC_SCRATCH_BYTES = 16 << 20

FP64, FP32, FP32_W16F, FP32_W16B = 0, 1, 2, 3
PLAN_GRAPH = 1
PLAN_AUTOTUNE = 2
PLAN_PROJECT = 4
PLAN_SYMMETRIC = 8
PLAN_PAIRS = 16
PLAN_FUSED = 32
PRECISIONS = {"f64": FP64, "f32": FP32, "f32-w16f": FP32_W16F, "f32-w16b": FP32_W16B}

TAIL_DTYPE = np.dtype([("segment", "<u4"), ("template", "<u4"), ("lag", "<u4"), ("rho", "<f4")])  # bfs_tail
TAIL64_DTYPE = np.dtype(
    [("segment", "<u4"), ("template", "<u4"), ("lag", "<u4"), ("reserved", "<u4"), ("rho", "<f8")]
)  # bfs_tail64
PEAK_DTYPE = np.dtype([("segment", "<u4"), ("lag", "<u4"), ("template", "<u4"), ("snr", "<f4")])
COINC_DTYPE = np.dtype([("pair", "<u4"), ("lag", "<u4"), ("template_a", "<u4"), ("template_b", "<u4"),
                        ("snr_a", "<f4"), ("snr_b", "<f4")])


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("n_min", ctypes.c_uint32),
        ("fs", ctypes.c_double),
        ("n_f0", ctypes.c_uint32),
        ("n_fdot", ctypes.c_uint32),
        ("f0_lo", ctypes.c_double),
        ("f0_hi", ctypes.c_double),
        ("fdot_lo", ctypes.c_double),
        ("fdot_hi", ctypes.c_double),
        ("n_tau", ctypes.c_uint32),
        ("tau", ctypes.POINTER(ctypes.c_double)),
        ("taper", ctypes.c_uint32),
        ("explicit_templates", ctypes.POINTER(ctypes.c_double)),
        ("n_explicit", ctypes.c_uint32),
        ("explicit_len", ctypes.c_uint32),
        ("kappa", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("tail_capacity", ctypes.c_uint64),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("device", ctypes.c_int),
        ("flags", ctypes.c_uint32),
        ("candidate", ctypes.c_uint32),
        ("tile", ctypes.c_uint32),
        ("kappa_hi", ctypes.c_double),
        ("coinc_delta_hz", ctypes.c_double),
    ]


class KernelInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("r1", ctypes.c_uint32),
        ("r2", ctypes.c_uint32),
        ("r3", ctypes.c_uint32),
        ("threads", ctypes.c_uint32),
        ("load_group", ctypes.c_uint32),
        ("split", ctypes.c_uint32),
        ("candidate", ctypes.c_uint32),
        ("n_candidates", ctypes.c_uint32),
        ("tuned_us", ctypes.c_float * 8),
        ("tile", ctypes.c_uint32),
        ("tile_us", ctypes.c_float * 5),
        ("fused", ctypes.c_uint32),
        ("fused_rows", ctypes.c_uint32),
        ("loop", ctypes.c_uint32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("m", ctypes.c_uint32),
        ("k", ctypes.c_uint32),
        ("threads_per_correlation", ctypes.c_uint32),
        ("bank_bytes", ctypes.c_uint64),
        ("plan_bytes", ctypes.c_uint64),
        ("precision", ctypes.c_uint32),
        ("n_min", ctypes.c_uint32),
        ("held_bytes", ctypes.c_uint64),
    ]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1708_01609_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sigs = {
        "bfsearch_plan": [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)],
        "bfsearch_filter": [vp, vp, vp, vp, u32, vp, ctypes.POINTER(vp)],
        "bfsearch_filter_noalloc": [vp, vp, u32, u32, vp, u64, vp, vp, vp],
        "bfsearch_fetch_tails": [vp, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "bfsearch_fetch_tails64": [vp, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "bfsearch_fetch_sigma": [vp, vp],
        "bfsearch_fetch_projection": [vp, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "bfsearch_fetch_coincidences": [vp, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "bfsearch_job_timing": [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
        "bfsearch_job_release": [vp],
        "bfsearch_job_poll": [vp, ctypes.POINTER(ctypes.c_int)],
        "bfsearch_plan_job_bytes": [vp, vp, u32, ctypes.POINTER(u64)],
        "bfsearch_destroy": [vp],
        "bfsearch_plan_get_info": [vp, ctypes.POINTER(PlanInfo)],
        "bfsearch_plan_kernel_info": [vp, u32, ctypes.POINTER(KernelInfo)],
        "bfsearch_correlate_dense": [vp, vp, u32, u32, vp, vp, vp],
        "bfsearch_correlate_dense_range": [vp, vp, u32, u32, u32, u32, vp, vp, vp],
        "bfsearch_plan_spectra": [vp, u32, u32, u32, vp, vp],
        "bfsearch_job_spectra": [vp, vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.bfsearch_status_string.argtypes = [ctypes.c_int]
    lib.bfsearch_status_string.restype = ctypes.c_char_p
    return lib


_lib = _load()


class BfsError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_lib.bfsearch_status_string(status).decode()} ({status})")


def _check(status: int, what: str) -> None:
    if status != BFS_OK:
        raise BfsError(status, what)


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


@dataclass
class Grid:
    """Chirp grid: template id j = i_f0 * n_fdot + i_fdot over inclusive linspaces."""

    n_f0: int
    n_fdot: int
    f0_range: tuple[float, float]
    fdot_range: tuple[float, float]
    taus: tuple[float, ...]
    taper: bool = True
    symmetric: bool = False   # chirp plus its time reversal


class Plan:
    """Resident template banks plus tables for the segment lengths n_min..n and one precision."""

    def __init__(self, n: int, fs: float, kappa: float, grid: Grid | None = None,
                 templates: np.ndarray | None = None, precision: str = "f32",
                 tail_capacity: int = 1 << 20, hbm_budget_bytes: int = 0, device: int = 0,
                 n_min: int | None = None, graph: bool = False, autotune: bool = False,
                 candidate: int = 0, tile: int = 0, project: bool = False, kappa_hi: float = 0.0,
                 pairs: bool = False, coinc_delta_hz: float = 0.0, fused: bool = False):
        d = PlanDesc()
        d.n, d.fs, d.kappa = int(n), float(fs), float(kappa)
        d.n_min = int(n_min) if n_min else 0
        d.precision = PRECISIONS[precision]
        d.tail_capacity, d.hbm_budget_bytes, d.device = int(tail_capacity), int(hbm_budget_bytes), int(device)
        d.flags = (PLAN_GRAPH if graph else 0) | (PLAN_AUTOTUNE if autotune else 0) | (PLAN_PROJECT if project else 0)
        d.candidate = int(candidate)
        d.tile = int(tile)
        d.kappa_hi = float(kappa_hi)
        d.coinc_delta_hz = float(coinc_delta_hz)
        if pairs:
            d.flags |= PLAN_PAIRS
        if fused:
            d.flags |= PLAN_FUSED
        self.pairs = bool(pairs)
        keep = []
        if templates is not None:
            t = np.ascontiguousarray(np.atleast_2d(np.asarray(templates, dtype=np.float64)))
            keep.append(t)
            d.explicit_templates = t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.n_explicit, d.explicit_len = t.shape
        else:
            if grid is None:
                raise ValueError("need a grid or explicit templates")
            taus = np.ascontiguousarray(np.asarray(grid.taus, dtype=np.float64))
            keep.append(taus)
            d.n_f0, d.n_fdot = int(grid.n_f0), int(grid.n_fdot)
            d.f0_lo, d.f0_hi = map(float, grid.f0_range)
            d.fdot_lo, d.fdot_hi = map(float, grid.fdot_range)
            d.n_tau = len(taus)
            d.tau = taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.taper = 1 if grid.taper else 0
            if grid.symmetric:
                d.flags |= PLAN_SYMMETRIC
        self.precision = precision
        self.sample_dtype = "float64" if precision == "f64" else "float32"
        # the record the kernels write (filter_noalloc's tail buffer), and fetch_tails' default
        self.tail_dtype = TAIL64_DTYPE if precision == "f64" else TAIL_DTYPE
        self.tail_capacity = int(tail_capacity)
        self.device = int(device)
        self._h = ctypes.c_void_p()
        _check(_lib.bfsearch_plan(ctypes.byref(d), ctypes.byref(self._h)), "bfsearch_plan")
        info = PlanInfo()
        _check(_lib.bfsearch_plan_get_info(self._h, ctypes.byref(info)), "bfsearch_plan_get_info")
        self.n, self.m, self.k, self.n_min = info.n, info.m, info.k, info.n_min
        self.threads_per_correlation = info.threads_per_correlation
        self.bank_bytes, self.plan_bytes = info.bank_bytes, info.plan_bytes

    def kernel_info(self, n: int | None = None) -> dict:
        """The fused kernel used at segment length n (default the largest): radices, workgroup
        size, load-group depth, split, chosen candidate and (autotuned plans) us per correlation."""
        ki = KernelInfo()
        _check(_lib.bfsearch_plan_kernel_info(self._h, int(n or 0), ctypes.byref(ki)), "bfsearch_plan_kernel_info")
        return {"n": ki.n, "radices": (ki.r1, ki.r2, ki.r3), "threads": ki.threads, "load_group": ki.load_group,
                "split": bool(ki.split), "candidate": ki.candidate, "n_candidates": ki.n_candidates,
                "tuned_us": [float(ki.tuned_us[i]) for i in range(ki.n_candidates)],
                "tile": ki.tile, "tile_us": {t: float(ki.tile_us[i]) for i, t in enumerate((1, 2, 4, 8, 16))},
                "fused": bool(ki.fused), "fused_rows": ki.fused_rows, "loop": bool(ki.loop)}

    def held_bytes(self) -> int:
        """Device bytes the plan holds now (plan memory, live jobs, pooled buffer sets)."""
        info = PlanInfo()
        _check(_lib.bfsearch_plan_get_info(self._h, ctypes.byref(info)), "bfsearch_plan_get_info")
        return int(info.held_bytes)

    def job_bytes(self, lengths) -> int:
        """Device bytes a filter call over segments of these lengths holds while live."""
        lens = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint32))
        out = ctypes.c_uint64()
        _check(_lib.bfsearch_plan_job_bytes(self._h, ctypes.c_void_p(lens.ctypes.data), int(lens.size),
                                            ctypes.byref(out)), "bfsearch_plan_job_bytes")
        return int(out.value)

    # ---------------------------------------------------------------- filter --
    def _check_tensor(self, y):
        import torch

        if not isinstance(y, torch.Tensor) or not y.is_cuda:
            raise TypeError("segments must be a CUDA tensor")
        want = torch.float64 if self.sample_dtype == "float64" else torch.float32
        if y.dtype != want:
            raise TypeError(f"segments must be {want}")
        if not y.is_contiguous():
            raise ValueError("segments must be contiguous")
        return y

    def _segments(self, y, n: int | None = None):
        n = self.n if n is None else int(n)
        y = self._check_tensor(y)
        if y.dim() == 1:
            y = y.unsqueeze(0)
        if y.dim() != 2 or y.shape[1] != n:
            raise ValueError(f"segments must have shape [S, {n}]")
        return y

    def filter(self, y, lengths=None, offsets=None, stream=None) -> "Job":
        """Queue the hot path after the work on `stream` (torch stream; default: current) and
        return the job.  The segment transforms run on `stream`, the fused kernels on the
        plan's stream paired with it (graph plans: all on `stream`); wait through the job
        (fetch, done, timing, release), not through `stream`.

        y: [S, n] for segments of the plan's largest length; or, with `lengths` (one power of
        two in [n_min, n] per segment), a flat tensor holding the segments back to back (or at
        element `offsets`).  Pair plans: pair p's two channels are segments 2p and 2p + 1."""
        if lengths is None:
            y = self._segments(y)
            S, lens_p, offs_p, lens = y.shape[0], None, None, [self.n] * y.shape[0]
        else:
            y = self._check_tensor(y)
            lens = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint32))
            S = int(lens.size)
            if offsets is None:
                offs = np.concatenate([[0], np.cumsum(lens[:-1], dtype=np.uint64)]).astype(np.uint64)
            else:
                offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
                if offs.size != S:
                    raise ValueError("offsets and lengths differ in size")
            if S and int(np.max(offs + lens.astype(np.uint64))) > y.numel():
                raise ValueError("a segment extends past the end of y")
            keep = (lens, offs)
            lens_p, offs_p = ctypes.c_void_p(lens.ctypes.data), ctypes.c_void_p(offs.ctypes.data)
            lens = [int(v) for v in lens]
        h = ctypes.c_void_p()
        _check(_lib.bfsearch_filter(self._h, ctypes.c_void_p(y.data_ptr()), offs_p, lens_p, S,
                                    _stream_handle(stream), ctypes.byref(h)), "bfsearch_filter")
        return Job(self, h, y, lens)

    def filter_noalloc(self, y, tails_out, count_out, sigma_out=None, stream=None) -> None:
        """The hot path with no allocation and no host synchronisation (bfsearch_filter_noalloc):
        queued on `stream` (default: current), returns at once.  y: [S, n_s] segments of one
        accepted length; tails_out: caller device memory for the unsorted tail records (a uint8
        tensor of capacity * tail_dtype.itemsize bytes); count_out: one int64 on the device, set to
        the exact tail count; sigma_out: [S, K] float64 on the device, or None.  Calls that overlap
        on one device share its scratch area and race; calls on one stream are ordered.  The
        records are the plan's tail_dtype (bfs_tail64 for FP64 plans, else bfs_tail)."""
        import torch

        y = self._check_tensor(y)
        if y.dim() == 1:
            y = y.unsqueeze(0)
        s, n = y.shape
        for t, dt in ((tails_out, torch.uint8), (count_out, torch.int64)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise TypeError(f"output buffers must be contiguous CUDA tensors of {dt}")
        if count_out.numel() < 1:
            raise ValueError("count_out needs one element")
        cap = tails_out.numel() // self.tail_dtype.itemsize
        sp = None
        if sigma_out is not None:
            if (not isinstance(sigma_out, torch.Tensor) or not sigma_out.is_cuda or sigma_out.dtype != torch.float64
                    or not sigma_out.is_contiguous() or sigma_out.numel() < s * self.k):
                raise TypeError("sigma_out must be a contiguous CUDA float64 tensor of S * K elements")
            sp = ctypes.c_void_p(sigma_out.data_ptr())
        _check(_lib.bfsearch_filter_noalloc(self._h, ctypes.c_void_p(y.data_ptr()), n, s,
                                            ctypes.c_void_p(tails_out.data_ptr()), cap,
                                            ctypes.c_void_p(count_out.data_ptr()), sp, _stream_handle(stream)),
               "bfsearch_filter_noalloc")

    def correlate_dense(self, y, first: int = 0, count: int | None = None, stream=None):
        """Diagnostic: every rho value [S, count, n_s] (plan sample dtype) and sigma [S, count]
        (float64) for segments y [S, n_s] of one accepted length n_s, against the templates
        first..first+count-1 (default: the whole bank)."""
        import torch

        y = self._check_tensor(y)
        if y.dim() == 1:
            y = y.unsqueeze(0)
        s, n = y.shape
        count = self.k - first if count is None else int(count)
        rho = torch.empty((s, count, n), dtype=y.dtype, device=y.device)
        sig = torch.empty((s, count), dtype=torch.float64, device=y.device)
        _check(_lib.bfsearch_correlate_dense_range(self._h, ctypes.c_void_p(y.data_ptr()), n, s, int(first), count,
                                                   ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                                   _stream_handle(stream)), "bfsearch_correlate_dense_range")
        return rho, sig

    def spectra(self, first: int = 0, count: int | None = None, n: int | None = None, stream=None):
        """Diagnostic: template spectra W_j[0..n/2] at segment length n (default the largest) as
        complex128, shape [count, n/2 + 1]."""
        import torch

        n = self.n if n is None else int(n)
        count = self.k - first if count is None else count
        out = torch.empty((count, n // 2 + 1, 2), dtype=torch.float64, device=f"cuda:{self.device}")
        _check(_lib.bfsearch_plan_spectra(self._h, n, first, count, ctypes.c_void_p(out.data_ptr()),
                                          _stream_handle(stream)), "bfsearch_plan_spectra")
        return torch.view_as_complex(out)

    def close(self) -> None:
        if self._h:
            _check(_lib.bfsearch_destroy(self._h), "bfsearch_destroy")
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                _lib.bfsearch_destroy(self._h)
        except Exception:
            pass


class Job:
    """One queued filter call; fetch results, then release (or use as a context manager)."""

    def __init__(self, plan: Plan, handle: ctypes.c_void_p, y, lengths):
        self.plan = plan
        self._h = handle
        self._y = y  # the device input stays alive until the job is released
        self.lengths = list(lengths)
        self.n_segments = len(self.lengths)

    def fetch_tails(self, capacity: int | None = None, allow_overflow: bool = False, wide: bool | None = None):
        """Tails sorted by (segment, template, lag), and the exact total: TAIL_DTYPE records (FP32
        rho), or with wide TAIL64_DTYPE (FP64 rho); the default is the plan's own record."""
        cap = self.plan.tail_capacity if capacity is None else int(capacity)
        wide = self.plan.tail_dtype is TAIL64_DTYPE if wide is None else bool(wide)
        out = np.empty(cap, dtype=TAIL64_DTYPE if wide else TAIL_DTYPE)  # the first n_written are filled
        nw, nt = ctypes.c_uint64(), ctypes.c_uint64()
        fetch = _lib.bfsearch_fetch_tails64 if wide else _lib.bfsearch_fetch_tails
        st = fetch(self._h, ctypes.c_void_p(out.ctypes.data), cap, ctypes.byref(nw), ctypes.byref(nt))
        if st == BFS_ERR_TAIL_OVERFLOW and allow_overflow:
            return out[: nw.value], nt.value
        _check(st, "bfsearch_fetch_tails")
        return out[: nw.value], nt.value

    def fetch_projection(self, capacity: int | None = None, allow_overflow: bool = False):
        """Per-lag max projection (projection plans): PEAK_DTYPE records sorted by (segment, lag), one
        per lag carrying a tail, and the exact number of such lags."""
        cap = sum(self.lengths) if capacity is None else int(capacity)
        out = np.empty(cap, dtype=PEAK_DTYPE)  # only the first n_written records are filled
        nw, nt = ctypes.c_uint64(), ctypes.c_uint64()
        st = _lib.bfsearch_fetch_projection(self._h, ctypes.c_void_p(out.ctypes.data), cap, ctypes.byref(nw),
                                            ctypes.byref(nt))
        if not (st == BFS_ERR_TAIL_OVERFLOW and allow_overflow):
            _check(st, "bfsearch_fetch_projection")
        return out[: nw.value], nt.value

    def fetch_coincidences(self, capacity: int | None = None, allow_overflow: bool = False):
        """Coincidences of detector pairs (plans with a coincidence window): COINC_DTYPE records
        sorted by (pair, lag), and the exact number found."""
        cap = sum(self.lengths[0::2]) if capacity is None else int(capacity)
        out = np.empty(cap, dtype=COINC_DTYPE)  # only the first n_written records are filled
        nw, nt = ctypes.c_uint64(), ctypes.c_uint64()
        st = _lib.bfsearch_fetch_coincidences(self._h, ctypes.c_void_p(out.ctypes.data), cap, ctypes.byref(nw),
                                              ctypes.byref(nt))
        if not (st == BFS_ERR_TAIL_OVERFLOW and allow_overflow):
            _check(st, "bfsearch_fetch_coincidences")
        return out[: nw.value], nt.value

    def done(self) -> bool:
        """True once every kernel of the job has finished (does not block)."""
        d = ctypes.c_int()
        _check(_lib.bfsearch_job_poll(self._h, ctypes.byref(d)), "bfsearch_job_poll")
        return bool(d.value)

    def fetch_sigma(self) -> np.ndarray:
        out = np.zeros((self.n_segments, self.plan.k), dtype=np.float64)
        _check(_lib.bfsearch_fetch_sigma(self._h, ctypes.c_void_p(out.ctypes.data)), "bfsearch_fetch_sigma")
        return out

    def timing(self) -> tuple[float, float]:
        """(fused correlation kernel ms, whole job ms) from HIP events on the streams the job's
        kernels run on."""
        c, t = ctypes.c_float(), ctypes.c_float()
        _check(_lib.bfsearch_job_timing(self._h, ctypes.byref(c), ctypes.byref(t)), "bfsearch_job_timing")
        return c.value, t.value

    def spectra(self):
        """Diagnostic: segment spectra Y_s[0..N_s/2] as complex128; [S, N/2 + 1] when every
        segment has the same length, else a list of 1-D tensors."""
        import torch

        sizes = [n // 2 + 1 for n in self.lengths]
        out = torch.empty((sum(sizes), 2), dtype=torch.float64, device=f"cuda:{self.plan.device}")
        _check(_lib.bfsearch_job_spectra(self._h, ctypes.c_void_p(out.data_ptr())), "bfsearch_job_spectra")
        c = torch.view_as_complex(out)
        if len(set(sizes)) == 1:
            return c.view(len(sizes), sizes[0])
        return list(torch.split(c, sizes))

    def release(self) -> None:
        if self._h:
            _check(_lib.bfsearch_job_release(self._h), "bfsearch_job_release")
            self._h = ctypes.c_void_p()
            self._y = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.release()


def tails_from_device(tails_out, count: int, dtype=TAIL_DTYPE) -> np.ndarray:
    """Decode the first min(count, capacity) records of a filter_noalloc tail buffer (a uint8 tensor)
    of the plan's tail_dtype into a numpy array, in device order."""
    cap = tails_out.numel() // dtype.itemsize
    n = min(int(count), cap)
    raw = tails_out[: n * dtype.itemsize].cpu().numpy()
    return raw.view(dtype).copy()


def status_string(status: int) -> str:
    return _lib.bfsearch_status_string(status).decode()


def raw_library() -> ctypes.CDLL:
    """The loaded C library (for tests of the ABI itself)."""
    return _lib
