"""CPU checks of the measurement's arithmetic and its one-GPU contract (no GPU needed)."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_flop_and_byte_counts_per_correlation():
    n = 1 << 16
    # the paper's FFT cost convention, 5 N log2 N (Eq. 10): 5.243 MFLOP at N = 2^16
    assert bench.nominal_flops(n) == 5 * n * 16 == 5242880
    # inverse real FFT 2.5 N log2 N, product 6 per bin over N/2 + 1 bins, threshold 1 per lag
    assert bench.algorithmic_flops(n) == 2.5 * n * 16 + 6 * (n // 2 + 1) + n == 2883590
    # one packed template row per correlation: N/2 complex values
    assert bench.algorithmic_bytes(n, 8) == 256 * 1024
    assert bench.algorithmic_bytes(n, 4) == 128 * 1024
    # fused synthesis adds the forward transform, the unpack and the synthesis of L samples
    extra = bench.fused_flops(n, 4096) - bench.algorithmic_flops(n)
    assert extra == 2.5 * n * 16 + 10 * (n // 2) + 20 * 4096
    for k in range(10, 18):
        assert bench.algorithmic_flops(1 << k) < bench.nominal_flops(1 << k)


def test_roofline_fractions_use_the_published_peaks():
    r = bench.roof(157.3e12, 8.0e12, 1.0)
    assert math.isclose(r["frac"], 1.0) and math.isclose(r["hbm_frac"], 1.0)
    assert math.isclose(r["achieved_tflops"], 157.3) and math.isclose(r["hbm_achieved_GBps"], 8000.0)
    # the C2 launch: 8192 correlations in 0.70 ms
    r = bench.roof(8192 * bench.algorithmic_flops(1 << 16), 8192 * bench.algorithmic_bytes(1 << 16, 8), 0.70e-3)
    assert 0.21 < r["frac"] < 0.22 and 0.38 < r["hbm_frac"] < 0.39


def test_measured_traffic_entries_are_plausible():
    # rocprofv3 bytes per C2 launch (8192 correlations): at least the algorithmic template
    # rows, at most 10 % more (segment row, twiddles, write-backs)
    for entry in bench.MEASURED_TRAFFIC.values():
        assert 2 * 2**30 <= entry["f32"] <= 1.1 * 2 * 2**30
        for key in ("f32-w16f", "f32-w16b"):
            assert 2**30 <= entry[key] <= 1.1 * 2**30
        assert entry["f32 fused"] < 1e8


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_exits_with_a_message(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       timeout=300, env=e, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
