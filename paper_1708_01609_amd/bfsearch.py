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

FP64, FP32, FP32_W16F, FP32_W16B = 0, 1, 2, 3
PRECISIONS = {"f64": FP64, "f32": FP32, "f32-w16f": FP32_W16F, "f32-w16b": FP32_W16B}

TAIL_DTYPE = np.dtype(
    [("segment", "<u4"), ("template", "<u4"), ("lag", "<u4"), ("reserved", "<u4"), ("rho", "<f8")]
)


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
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
        ("reserved", ctypes.c_uint32),
    ]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1708_01609_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sigs = {
        "bfsearch_plan": [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)],
        "bfsearch_filter": [vp, vp, u32, vp, ctypes.POINTER(vp)],
        "bfsearch_fetch_tails": [vp, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "bfsearch_fetch_sigma": [vp, vp],
        "bfsearch_job_timing": [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
        "bfsearch_job_release": [vp],
        "bfsearch_destroy": [vp],
        "bfsearch_plan_get_info": [vp, ctypes.POINTER(PlanInfo)],
        "bfsearch_correlate_dense": [vp, vp, u32, vp, vp, vp],
        "bfsearch_plan_spectra": [vp, u32, u32, vp, vp],
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


class Plan:
    """Resident template bank plus tables for one segment length and precision."""

    def __init__(self, n: int, fs: float, kappa: float, grid: Grid | None = None,
                 templates: np.ndarray | None = None, precision: str = "f32",
                 tail_capacity: int = 1 << 20, hbm_budget_bytes: int = 0, device: int = 0):
        d = PlanDesc()
        d.n, d.fs, d.kappa = int(n), float(fs), float(kappa)
        d.precision = PRECISIONS[precision]
        d.tail_capacity, d.hbm_budget_bytes, d.device = int(tail_capacity), int(hbm_budget_bytes), int(device)
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
        self.precision = precision
        self.sample_dtype = "float64" if precision == "f64" else "float32"
        self.tail_capacity = int(tail_capacity)
        self.device = int(device)
        self._h = ctypes.c_void_p()
        _check(_lib.bfsearch_plan(ctypes.byref(d), ctypes.byref(self._h)), "bfsearch_plan")
        info = PlanInfo()
        _check(_lib.bfsearch_plan_get_info(self._h, ctypes.byref(info)), "bfsearch_plan_get_info")
        self.n, self.m, self.k = info.n, info.m, info.k
        self.threads_per_correlation = info.threads_per_correlation
        self.bank_bytes, self.plan_bytes = info.bank_bytes, info.plan_bytes

    # ---------------------------------------------------------------- filter --
    def _segments(self, y):
        import torch

        if not isinstance(y, torch.Tensor) or not y.is_cuda:
            raise TypeError("segments must be a CUDA tensor")
        if y.dim() == 1:
            y = y.unsqueeze(0)
        if y.dim() != 2 or y.shape[1] != self.n:
            raise ValueError(f"segments must have shape [S, {self.n}]")
        want = torch.float64 if self.sample_dtype == "float64" else torch.float32
        if y.dtype != want:
            raise TypeError(f"segments must be {want}")
        return y.contiguous()

    def filter(self, y, stream=None) -> "Job":
        """Queue the hot path on `stream` (torch stream; default: current) and return the job."""
        y = self._segments(y)
        h = ctypes.c_void_p()
        _check(_lib.bfsearch_filter(self._h, ctypes.c_void_p(y.data_ptr()), y.shape[0],
                                    _stream_handle(stream), ctypes.byref(h)), "bfsearch_filter")
        return Job(self, h, y)

    def correlate_dense(self, y, stream=None):
        """Diagnostic: every rho value [S, K, N] (plan sample dtype) and sigma [S, K] (float64)."""
        import torch

        y = self._segments(y)
        s = y.shape[0]
        rho = torch.empty((s, self.k, self.n), dtype=y.dtype, device=y.device)
        sig = torch.empty((s, self.k), dtype=torch.float64, device=y.device)
        _check(_lib.bfsearch_correlate_dense(self._h, ctypes.c_void_p(y.data_ptr()), s,
                                             ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(sig.data_ptr()),
                                             _stream_handle(stream)), "bfsearch_correlate_dense")
        return rho, sig

    def spectra(self, first: int = 0, count: int | None = None, stream=None):
        """Diagnostic: template spectra W_j[0..N/2] as complex128, shape [count, N/2 + 1]."""
        import torch

        count = self.k - first if count is None else count
        out = torch.empty((count, self.m + 1, 2), dtype=torch.float64, device=f"cuda:{self.device}")
        _check(_lib.bfsearch_plan_spectra(self._h, first, count, ctypes.c_void_p(out.data_ptr()),
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

    def __init__(self, plan: Plan, handle: ctypes.c_void_p, y):
        self.plan = plan
        self._h = handle
        self._y = y  # the device input stays alive until the job is released
        self.n_segments = y.shape[0]

    def fetch_tails(self, capacity: int | None = None, allow_overflow: bool = False):
        """Tails sorted by (segment, template, lag) as a TAIL_DTYPE array, and the exact total."""
        cap = self.plan.tail_capacity if capacity is None else int(capacity)
        out = np.zeros(cap, dtype=TAIL_DTYPE)
        nw, nt = ctypes.c_uint64(), ctypes.c_uint64()
        st = _lib.bfsearch_fetch_tails(self._h, ctypes.c_void_p(out.ctypes.data), cap, ctypes.byref(nw),
                                       ctypes.byref(nt))
        if st == BFS_ERR_TAIL_OVERFLOW and allow_overflow:
            return out[: nw.value], nt.value
        _check(st, "bfsearch_fetch_tails")
        return out[: nw.value], nt.value

    def fetch_sigma(self) -> np.ndarray:
        out = np.zeros((self.n_segments, self.plan.k), dtype=np.float64)
        _check(_lib.bfsearch_fetch_sigma(self._h, ctypes.c_void_p(out.ctypes.data)), "bfsearch_fetch_sigma")
        return out

    def timing(self) -> tuple[float, float]:
        """(fused correlation kernel ms, whole job ms) from HIP events on the job's stream."""
        c, t = ctypes.c_float(), ctypes.c_float()
        _check(_lib.bfsearch_job_timing(self._h, ctypes.byref(c), ctypes.byref(t)), "bfsearch_job_timing")
        return c.value, t.value

    def spectra(self):
        """Diagnostic: segment spectra Y_s[0..N/2] as complex128 [S, N/2 + 1]."""
        import torch

        out = torch.empty((self.n_segments, self.plan.m + 1, 2), dtype=torch.float64,
                          device=f"cuda:{self.plan.device}")
        _check(_lib.bfsearch_job_spectra(self._h, ctypes.c_void_p(out.data_ptr())), "bfsearch_job_spectra")
        return torch.view_as_complex(out)

    def release(self) -> None:
        if self._h:
            _check(_lib.bfsearch_job_release(self._h), "bfsearch_job_release")
            self._h = ctypes.c_void_p()
            self._y = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.release()


def status_string(status: int) -> str:
    return _lib.bfsearch_status_string(status).decode()


def raw_library() -> ctypes.CDLL:
    """The loaded C library (for tests of the ABI itself)."""
    return _lib
