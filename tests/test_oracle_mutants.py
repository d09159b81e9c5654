"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that the pins catch each.

Every mutant is a one-line source edit of oracle/bfsearch_oracle.py, loaded as a
separate module; the pin functions of test_oracle_pins are then run against it
and at least one of them must fail.
"""
import importlib.util
import os
import sys
import types

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "bfsearch_oracle.py")

MUTANTS = {
    "conj_on_segment": ("np.conj(wt) * yt", "wt * np.conj(yt)"),
    "irfft_scaled": ("return sfft.irfft(np.conj(wt) * yt, n=n, axis=-1, workers=_workers())",
                     "return 2.0 * sfft.irfft(np.conj(wt) * yt, n=n, axis=-1, workers=_workers())"),
    "sigma_n_minus_1": ("np.sum(rho * rho, axis=-1) / rho.shape[-1]", "np.sum(rho * rho, axis=-1) / (rho.shape[-1] - 1)"),
    "parseval_no_factor2": ("+ 2.0 * np.sum(p[..., 1:n // 2], axis=-1)", "+ np.sum(p[..., 1:n // 2], axis=-1)"),
    "parseval_drops_dc": ("s = p[..., 0] + p[..., n // 2] +", "s = p[..., n // 2] +"),
    "threshold_ge": ("np.abs(rho) > kappa * sigma", "np.abs(rho) >= kappa * sigma"),
    "threshold_no_abs": ("keep = np.abs(rho) > kappa * sigma", "keep = rho > kappa * sigma"),
    "chirp_no_half": ("cycles = f0 * t + 0.5 * fdot * t * t", "cycles = f0 * t + fdot * t * t"),
    "chirp_fdot_sign": ("cycles = f0 * t + 0.5 * fdot * t * t", "cycles = f0 * t - 0.5 * fdot * t * t"),
    "hann_periodic": ("np.cos(2.0 * np.pi * m / (length - 1))", "np.cos(2.0 * np.pi * m / length)"),
    "grid_fdot_major": ("return f0s[j // int(n_fdot)], fds[j % int(n_fdot)]",
                        "return f0s[j % int(n_f0)], fds[j // int(n_f0)]"),
    "no_normalisation": ("w = w / np.sqrt(e)", "w = w / e"),
    "direct_lag_reversed": ("rho += w[m] * np.roll(y, -m)", "rho += w[m] * np.roll(y, m)"),
    "symmetric_not_added": ("w = w + w[::-1]", "w = w[::-1]"),
    "band_inclusive": ("keep &= np.abs(rho) < kappa_hi * sigma", "keep &= np.abs(rho) <= kappa_hi * sigma"),
    "projection_raw_rho": ("v = abs(r) / float(sigma[s, j])", "v = abs(r)"),
    "projection_signed": ("v = abs(r) / float(sigma[s, j])", "v = r / float(sigma[s, j])"),
    "projection_highest_id": ("if v > bv or (v == bv and j < bj):", "if v > bv or (v == bv and j > bj):"),
    "coinc_window_inclusive": ("if abs(f0[ja] - f0[jb]) < delta:", "if abs(f0[ja] - f0[jb]) <= delta:"),
    "coinc_no_abs": ("if abs(f0[ja] - f0[jb]) < delta:", "if f0[ja] - f0[jb] < delta:"),
    "coinc_template_ids": ("if abs(f0[ja] - f0[jb]) < delta:", "if abs(ja - jb) < delta:"),
    "coinc_pair_from_segment": ("(first if int(s) % 2 == 0 else second)[(int(s) // 2, int(n))] = (int(j), float(v))",
                                "(first if int(s) % 2 == 0 else second)[(int(s), int(n))] = (int(j), float(v))"),
    "coinc_snr_swapped": ("rows.append((key[0], key[1], ja, jb, va, vb))", "rows.append((key[0], key[1], ja, jb, vb, va))"),
}

PIN_TESTS = [
    (pins.test_fft_and_direct_match_brute_force, [(64, 16), (256, 3)]),
    (pins.test_impulse_closed_form, [(5,)]),
    (pins.test_rectangular_template_tone_closed_form, [(37, 1000, 0.7)]),
    (pins.test_parseval_identity_any_input, [()]),
    (pins.test_eq7_equals_parseval_for_bandlimited_only, [()]),
    (pins.test_hann_is_numpy_symmetric_hann, [()]),
    (pins.test_chirp_quarter_rate_tone_exact, [()]),
    (pins.test_chirp_instantaneous_frequency, [(600.0, 300.0)]),
    (pins.test_template_unit_energy_and_grid_order, [()]),
    (pins.test_cauchy_schwarz_recovers_noise_free_injection, [()]),
    (pins.test_threshold_strict_and_absolute, [()]),
    (pins.test_search_tails_equal_brute_force_threshold, [()]),
    (pins.test_sigma_expectation_equals_inband_template_energy, [()]),
    (pins.test_max_projection_equals_brute_force_argmax, [()]),
    (pins.test_max_projection_ties_scale_and_sign, [()]),
    (pins.test_time_symmetric_template_mirrors_correlation_of_reversed_data, [()]),
    (pins.test_band_threshold_keeps_only_the_band, [()]),
    (pins.test_coincidences_of_table3_rows, [(50.0, [17713196, 17713197, 17713198, 17713199]),
                                             (5.0, [17713197, 17713198, 17713199]), (1.0, [])]),
    (pins.test_coincidences_of_identical_channels_are_every_projected_lag, [()]),
    (pins.test_coincidences_swap_symmetry_and_monotone_window, [()]),
]


def _load_mutant(name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mod = types.ModuleType(f"oracle_mutant_{name}")
    mod.__file__ = SRC
    exec(compile(src.replace(old, new, 1), SRC, "exec"), mod.__dict__)
    return mod


def _pins_fail(monkeypatch, mod):
    for attr in oracle.__all__:
        monkeypatch.setattr(oracle, attr, getattr(mod, attr))
    for fn, cases in PIN_TESTS:
        for args in cases:
            try:
                fn(*args)
            except AssertionError:
                return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(monkeypatch, name):
    old, new = MUTANTS[name]
    mod = _load_mutant(name, old, new)
    assert _pins_fail(monkeypatch, mod), f"no pin fails for mutant {name}"


def test_unmutated_copy_passes_all_pins(monkeypatch):
    mod = _load_mutant("identity", "import os", "import os")
    assert not _pins_fail(monkeypatch, mod)
