"""Spectra of probe records (Sec. 3.2: velocity and pressure recorded at every step at
points on the burner axis; the precessing-vortex-core frequency is read off their
spectra).  Post-processing on the host: the records come from lbm_set_probes."""
import numpy as np


def power_spectrum(series, dt=1.0):
    """One-sided power spectral density of a record (last axis = time) after removing its
    mean, with a Hann window; returns (frequencies in 1/dt units, PSD)."""
    x = np.asarray(series, dtype=np.float64)
    x = x - x.mean(axis=-1, keepdims=True)
    n = x.shape[-1]
    w = np.hanning(n)
    X = np.fft.rfft(x * w, axis=-1)
    psd = (np.abs(X) ** 2) * 2.0 * dt / (w * w).sum()
    psd[..., 0] /= 2.0
    if n % 2 == 0:
        psd[..., -1] /= 2.0
    return np.fft.rfftfreq(n, dt), psd


def dominant_frequency(series, dt=1.0):
    """Frequency of the largest spectral peak (excluding zero), refined by a parabola
    through the peak bin and its neighbours."""
    f, p = power_spectrum(series, dt)
    k = 1 + int(np.argmax(p[..., 1:]))
    if 1 <= k < len(f) - 1:
        a, b, c = np.log(p[k - 1]), np.log(p[k]), np.log(p[k + 1])
        shift = 0.5 * (a - c) / (a - 2 * b + c)
        return float(f[k] + shift * (f[1] - f[0]))
    return float(f[k])
