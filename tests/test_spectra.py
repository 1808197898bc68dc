"""Host-side probe spectra: the peak of a sampled sinusoid in noise is at its frequency
and Parseval's relation holds for the one-sided density."""
import numpy as np

from paper_2207_11567_amd.spectra import dominant_frequency, power_spectrum


def test_sinusoid_peak_and_parseval():
    dt, n = 5e-8, 4096
    t = np.arange(n) * dt
    f0 = 516.4 * 1e3 / 10.0                     # a frequency between bins
    rng = np.random.default_rng(3)
    x = 0.7 * np.sin(2 * np.pi * f0 * t) + 0.01 * rng.standard_normal(n)
    assert abs(dominant_frequency(x, dt) / f0 - 1) < 2e-3
    y = rng.standard_normal(n)
    f, p = power_spectrum(y, dt)
    w = np.hanning(n)
    yw = (y - y.mean()) * w
    assert abs(p.sum() * (f[1] - f[0]) / ((yw ** 2).sum() / (w * w).sum()) - 1) < 1e-12
