"""C-ABI checks that need no GPU: exported symbols and host-side argument validation.

Every invalid call below must be rejected before the library makes any HIP
call, so these run on a machine without a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfsearch.h")


@pytest.fixture(scope="module")
def bfs():
    from paper_1708_01609_amd import build as b

    if not os.path.exists(b.LIB):
        b.build()
    from paper_1708_01609_amd import bfsearch

    return bfsearch


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:bfs_status|const char\*)\s+(bfsearch_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bfsearch_plan", "bfsearch_filter", "bfsearch_fetch_tails", "bfsearch_fetch_sigma",
                     "bfsearch_job_release", "bfsearch_destroy", "bfsearch_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol(bfs):
    lib = bfs.raw_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header(bfs):
    assert ctypes.sizeof(bfs.PlanInfo) == 48
    assert bfs.TAIL_DTYPE.itemsize == 16 and bfs.TAIL64_DTYPE.itemsize == 24
    assert bfs.PEAK_DTYPE.itemsize == 16
    assert bfs.COINC_DTYPE.itemsize == 24
    # bfs_plan_desc field order as declared (spot-check offsets of the 64-bit fields)
    assert bfs.PlanDesc.fs.offset == 8
    assert bfs.PlanDesc.tail_capacity.offset % 8 == 0


def test_status_strings(bfs):
    assert bfs.status_string(0) == "ok"
    assert "overflow" in bfs.status_string(-4)
    assert bfs.status_string(-99) == "unknown status"


def _desc(bfs, **kw):
    d = bfs.PlanDesc()
    taus = np.array([1.0])
    d.n, d.fs, d.n_f0, d.n_fdot = 1 << 16, 4096.0, 4, 4
    d.f0_lo, d.f0_hi, d.fdot_lo, d.fdot_hi = 350.0, 2000.0, -500.0, 500.0
    d.n_tau = 1
    d.tau = taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.taper, d.kappa, d.precision, d.tail_capacity = 1, 5.0, bfs.FP32, 1024
    for k, v in kw.items():
        setattr(d, k, v)
    return d, taus


@pytest.mark.parametrize("field,value", [
    ("n", 1000),            # not a power of two
    ("n", 0),
    ("fs", 0.0),
    ("fs", -1.0),
    ("kappa", -1.0),
    ("tail_capacity", 0),
    ("precision", 7),
    ("taper", 2),
    ("n_f0", 0),
    ("n_tau", 0),
    ("fdot_hi", float("nan")),
    ("n_min", 3000),        # not a power of two
    ("n_min", 1 << 17),     # above n
    ("n_min", 2048),        # shorter than the 4096-sample templates
    ("flags", 64),          # unknown flag
    ("kappa_hi", 4.0),      # band edge below kappa
    ("kappa_hi", float("inf")),
    ("candidate", 99),      # no such kernel candidate
    ("tile", 1 << 20),      # tile beyond the segment limit
    ("coinc_delta_hz", 50.0),  # a coincidence window without pairs and projection
    ("coinc_delta_hz", -1.0),
    ("coinc_delta_hz", float("nan")),
])
def test_plan_rejects_invalid_descriptor(bfs, field, value):
    d, keep = _desc(bfs, **{field: value})
    out = ctypes.c_void_p(1)
    st = bfs.raw_library().bfsearch_plan(ctypes.byref(d), ctypes.byref(out))
    assert st == bfs.BFS_ERR_INVALID_ARG
    assert not out.value


def test_plan_desc_layout_matches_header(bfs):
    # field offsets a C compiler gives bfs_plan_desc on x86-64 (natural alignment)
    off = {f: getattr(bfs.PlanDesc, f).offset for f, _ in bfs.PlanDesc._fields_}
    assert off["n"] == 0 and off["n_min"] == 4 and off["fs"] == 8
    assert off["flags"] == off["device"] + 4 and off["candidate"] == off["flags"] + 4
    assert off["tile"] == off["candidate"] + 4 and off["kappa_hi"] % 8 == 0 and off["kappa_hi"] > off["tile"]
    assert ctypes.sizeof(bfs.PlanDesc) % 8 == 0
    assert ctypes.sizeof(bfs.KernelInfo) == 9 * 4 + 8 * 4 + 4 + 5 * 4 + 3 * 4


def test_fused_plans_are_checked_on_the_host(bfs):
    # fused synthesis needs grid templates, FP32 precision, single segments and a length with a
    # fused kernel (2^10, 2^13, 2^16); anything else is refused before the device is touched
    lib = bfs.raw_library()
    cases = [dict(n=1 << 16, precision=bfs.FP64), dict(n=1 << 14), dict(n=1 << 17),
             dict(n=1 << 16, flags=bfs.PLAN_PAIRS)]
    for kw in cases:
        flags = bfs.PLAN_FUSED | kw.pop("flags", 0)
        d, keep = _desc(bfs, flags=flags, **kw)
        taus = np.array([0.1])
        d.tau = taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        out = ctypes.c_void_p()
        assert lib.bfsearch_plan(ctypes.byref(d), ctypes.byref(out)) == bfs.BFS_ERR_UNSUPPORTED, kw
    temps = np.ones((2, 16))
    d, keep = _desc(bfs, n=1 << 16, flags=bfs.PLAN_FUSED)
    d.explicit_templates = temps.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.n_explicit, d.explicit_len = 2, 16
    out = ctypes.c_void_p()
    assert lib.bfsearch_plan(ctypes.byref(d), ctypes.byref(out)) == bfs.BFS_ERR_UNSUPPORTED


def test_noalloc_arguments_are_checked_on_the_host(bfs):
    lib = bfs.raw_library()
    count = ctypes.c_uint64()
    assert lib.bfsearch_filter_noalloc(None, ctypes.c_void_p(16), 0, 1, None, 0, ctypes.byref(count), None,
                                       None) == bfs.BFS_ERR_INVALID_ARG
    assert "scratch" in bfs.status_string(bfs.BFS_ERR_SCRATCH_LIMIT)


def test_plan_rejects_template_longer_than_segment(bfs):
    taus = np.array([2.0])  # 8192 samples > N = 4096
    d, _ = _desc(bfs, n=4096)
    d.tau = taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = ctypes.c_void_p()
    assert bfs.raw_library().bfsearch_plan(ctypes.byref(d), ctypes.byref(out)) == bfs.BFS_ERR_INVALID_ARG


def test_pair_plans_need_pairs_and_projection_for_a_window(bfs):
    # a window needs pairs and projection together, and grid templates (their initial frequencies)
    for flags in (bfs.PLAN_PAIRS, bfs.PLAN_PROJECT):
        d, keep = _desc(bfs, flags=flags, coinc_delta_hz=50.0)
        out = ctypes.c_void_p()
        assert bfs.raw_library().bfsearch_plan(ctypes.byref(d), ctypes.byref(out)) == bfs.BFS_ERR_INVALID_ARG
    temps = np.ones((2, 16))
    d, keep = _desc(bfs, flags=bfs.PLAN_PAIRS | bfs.PLAN_PROJECT, coinc_delta_hz=50.0)
    d.explicit_templates = temps.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.n_explicit, d.explicit_len = 2, 16
    out = ctypes.c_void_p()
    assert bfs.raw_library().bfsearch_plan(ctypes.byref(d), ctypes.byref(out)) == bfs.BFS_ERR_INVALID_ARG


def test_plan_reports_unsupported_sizes(bfs):
    # pairs at lengths whose transform is split (2^17 FP32, 2^14 FP64) are not built
    for n, prec in ((1 << 17, bfs.FP32), (1 << 14, bfs.FP64)):
        d, keep = _desc(bfs, n=n, precision=prec, flags=bfs.PLAN_PAIRS)
        taus = np.array([0.1])
        d.tau = taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        out = ctypes.c_void_p()
        assert bfs.raw_library().bfsearch_plan(ctypes.byref(d), ctypes.byref(out)) == bfs.BFS_ERR_UNSUPPORTED
    for n, prec in ((1 << 18, bfs.FP32), (1 << 15, bfs.FP64), (1 << 9, bfs.FP32)):
        d, keep = _desc(bfs, n=n, precision=prec)
        taus = np.array([0.1])
        d.tau = taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        out = ctypes.c_void_p()
        assert bfs.raw_library().bfsearch_plan(ctypes.byref(d), ctypes.byref(out)) == bfs.BFS_ERR_UNSUPPORTED


def test_null_handles_are_rejected(bfs):
    lib = bfs.raw_library()
    out = ctypes.c_void_p()
    nw, nt = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.bfsearch_plan(None, ctypes.byref(out)) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_filter(None, None, None, None, 1, None, ctypes.byref(out)) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_fetch_tails(None, None, 0, ctypes.byref(nw), ctypes.byref(nt)) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_fetch_sigma(None, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_job_release(None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_destroy(None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_correlate_dense(None, None, 0, 1, None, None, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_correlate_dense_range(None, None, 0, 1, 0, 1, None, None, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_plan_spectra(None, 0, 0, 1, None, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_job_spectra(None, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_job_timing(None, None, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_plan_get_info(None, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_plan_kernel_info(None, 0, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_job_poll(None, None) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_fetch_projection(None, None, 0, ctypes.byref(nw), ctypes.byref(nt)) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_fetch_coincidences(None, None, 0, ctypes.byref(nw), ctypes.byref(nt)) == bfs.BFS_ERR_INVALID_ARG
    assert lib.bfsearch_plan_job_bytes(None, None, 1, None) == bfs.BFS_ERR_INVALID_ARG
