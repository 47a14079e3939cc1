"""Oracle: matched-filter SNR series and template norm (section II.A).

Discretisation of equation (matched_filter) on a segment of n samples at
rate fs (T = n / fs, df = 1 / T, f_j = j df):

    N_h^2 = 4 df sum_{j in B} |h~_j|^2 / S_j                  (norm)
    Y_j   = (4 df / N_h) x~_j conj(h~_j) / S_j   for j in B,  0 otherwise
    z[m]  = sum_{j=0}^{n-1} Y_j exp(+2 pi i j m / n)          (complex SNR)

where B = {j : f_low <= f_j <= f_high} is the band of the PSD-infinite
convention, and every negative-frequency bin of Y is zero (the integral of
equation (matched_filter) runs over f >= 0 only).  z[m] is the SNR for
coalescence time m / fs, circular in the segment.
"""
from __future__ import annotations

import numpy as np

from . import taylorf2


def band_mask(fs: float, n: int, f_low: float, f_high: float) -> np.ndarray:
    """Boolean mask over bins j = 0..n/2 of f_low <= f_j <= f_high."""
    f = np.arange(n // 2 + 1, dtype=np.float64) * (fs / n)
    return (f >= f_low) & (f <= f_high)


def template_spectrum(fs: float, n: int, m1: float, m2: float) -> np.ndarray:
    """h~_j for j = 0..n/2 (complex128)."""
    f = np.arange(n // 2 + 1, dtype=np.float64) * (fs / n)
    return taylorf2.template(f, m1, m2)


def norm(fs: float, n: int, f_low: float, f_high: float, psd: np.ndarray,
         h: np.ndarray) -> float:
    """N_h = sqrt(4 df sum_B |h~|^2 / S) (normalisation after eq. matched_filter)."""
    band = band_mask(fs, n, f_low, f_high)
    df = fs / n
    return float(np.sqrt(4.0 * df * np.sum(np.abs(h[band]) ** 2 / psd[band])))


def snr_spectrum(fs, n, f_low, f_high, xf, psd, h):
    """Y_j over the full n-point frequency axis, and N_h."""
    band = band_mask(fs, n, f_low, f_high)
    nh = norm(fs, n, f_low, f_high, psd, h)
    y = np.zeros(n, dtype=np.complex128)
    idx = np.nonzero(band)[0]
    y[idx] = (4.0 * (fs / n) / nh) * xf[idx] * np.conj(h[idx]) / psd[idx]
    return y, nh


def snr_series(fs, n, f_low, f_high, xf, psd, m1, m2):
    """Complex SNR z[m], m = 0..n-1, of template (m1, m2), and its norm N_h.

    The inverse transform is a library FFT: z = n * ifft(Y).
    """
    h = template_spectrum(fs, n, m1, m2)
    y, nh = snr_spectrum(fs, n, f_low, f_high, xf, psd, h)
    return n * np.fft.ifft(y), nh


def snr_series_bruteforce(fs, n, f_low, f_high, xf, psd, m1, m2):
    """The same sum written out term by term, O(n^2); for n of a few thousand."""
    h = template_spectrum(fs, n, m1, m2)
    y, nh = snr_spectrum(fs, n, f_low, f_high, xf, psd, h)
    j = np.nonzero(y)[0]
    m = np.arange(n)
    phase = np.exp(2j * np.pi * np.outer(m, j) / n)
    return phase @ y[j], nh


def grid_snr_series(grid, xf, psd, m1, m2):
    """snr_series for a grid-like object with fs, n, f_low, f_high."""
    return snr_series(grid.fs, grid.n, grid.f_low, grid.f_high, xf, psd, m1, m2)
