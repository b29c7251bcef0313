"""Host-side analysis of the benchmark harness (no GPU)."""
import numpy as np

import bench


def test_main_frequency_finds_the_dominant_peak_over_a_trend():
    # E_k-like signal: a slow drift, a main oscillation and a weaker harmonic
    t = np.arange(0, 1000, 0.02)
    ek = 0.046 + 1e-6 * (t / 1000) ** 2 + 1e-5 * np.sin(2 * np.pi * 0.6144 * t) + 3e-6 * np.sin(2 * np.pi * 1.2288 * t)
    f, res, osc = bench.main_frequency(t, ek)
    assert abs(f - 0.6144) <= res
    assert 1e-4 < osc < 3e-4


def test_main_frequency_removes_a_quadratic_drift_exactly():
    # the detrending is a quadratic fit: a drift alone leaves no oscillation
    t = np.arange(750, 1500, 0.02)
    ek = 0.0416 - 2e-6 * (t - 1000) / 500 + 3e-7 * ((t - 1000) / 500) ** 2
    _, _, osc = bench.main_frequency(t, ek)
    assert osc < 1e-12
