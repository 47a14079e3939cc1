"""Oracle: ratio kernels, truncation and reconstruction (sections II.B-II.D,
appendix A).

Ratio waveform (equation ratio_waveform) with the window of equation (window):

    R~_j = W(f_j) (B_k / B_ref)(f_j) exp(-i (Psi_k - Psi_ref)(f_j)),  j = 0..n_r/2
    w    = inverse real DFT of R~ over n_r points (Hermitian extension),
    r(t_m) = fs * w[m]   [1/s]

so that (equation convolution, discretised on the circular segment of n = n_r
samples, the convention under which it reproduces equation related_binning
exactly)

    z_k[m] = (N_ref / N_k) sum_s z_ref[(m + s) mod n] w[s mod n_r].

Taper widths (section II.C): df_low = |dtau'(f_low)|^(-1/2) capped at
df_low_max (5 Hz) and set to the cap when dtau' = 0; df_high = 53 Hz; here
dtau = tau_k - tau_ref with tau(f) the time from f to merger, so
|dtau'| = |t_k'(f) - t_ref'(f)|.

Truncation (section II.D): the kernel is kept on the contiguous signed index
range [m_lo, m_hi] spanning every tap with |r(t_m)| >= threshold (threshold
in 1/s, 1e-3 in the paper); taps in between are all kept.  The appendix-A
analytic window is returned separately as a containment check.
"""
from __future__ import annotations

import math

import numpy as np

from . import taylorf2


def window(f, f_low, f_high, df_low, df_high) -> np.ndarray:
    """W(f) of equation (window): cosine tapers below f_low and above f_high."""
    f = np.asarray(f, dtype=np.float64)
    w = np.zeros(f.shape, dtype=np.float64)
    lo = (f > f_low - df_low) & (f < f_low)
    w[lo] = 0.5 * (1.0 + np.cos(math.pi * (f[lo] - f_low) / df_low))
    w[(f >= f_low) & (f <= f_high)] = 1.0
    hi = (f > f_high) & (f < f_high + df_high)
    w[hi] = 0.5 * (1.0 - np.cos(math.pi * (f[hi] - (f_high + df_high)) / df_high))
    return w


def dtau_prime(f, ref, tgt) -> float:
    """d/df [tau_tgt - tau_ref](f) [s/Hz] (section II.C)."""
    return float(-(taylorf2.dtime_dfrequency(f, *tgt) - taylorf2.dtime_dfrequency(f, *ref)))


def df_low(f_low, ref, tgt, df_low_max=5.0) -> float:
    """Lower taper width: min(df_low_max, |dtau'(f_low)|^(-1/2)), the cap when dtau' = 0."""
    d = abs(dtau_prime(f_low, ref, tgt))
    if d == 0.0:
        return df_low_max
    return min(df_low_max, 1.0 / math.sqrt(d))


def ratio_spectrum(fs, n_r, f_low, f_high, df_lo, df_hi, ref, tgt) -> np.ndarray:
    """R~_j, j = 0..n_r/2 (complex128), zero where W = 0."""
    f = np.arange(n_r // 2 + 1, dtype=np.float64) * (fs / n_r)
    wdw = window(f, f_low, f_high, df_lo, df_hi)
    out = np.zeros(f.shape, dtype=np.complex128)
    on = wdw > 0
    amp = taylorf2.amplitude(f[on], *tgt) / taylorf2.amplitude(f[on], *ref)
    dpsi = taylorf2.phase(f[on], *tgt) - taylorf2.phase(f[on], *ref)
    out[on] = wdw[on] * amp * np.exp(-1j * dpsi)
    return out


def ratio_taps(fs, n_r, f_low, f_high, df_lo, df_hi, ref, tgt) -> np.ndarray:
    """Untruncated real kernel w[m], m = 0..n_r-1 (library inverse real FFT)."""
    return np.fft.irfft(ratio_spectrum(fs, n_r, f_low, f_high, df_lo, df_hi, ref, tgt), n_r)


def truncate(w: np.ndarray, fs: float, threshold: float, per_second: bool = True):
    """Contiguous signed support of |r| >= threshold.

    threshold is in 1/s on r = fs * w (the paper's unit) when per_second, else
    on w itself.  Signed index s in (-n_r/2, n_r/2] stands for sample s mod n_r.
    Returns (m_lo, taps) with taps = w[m_lo .. m_hi] (length 0 when nothing
    reaches the threshold, with m_lo = 0).
    """
    n_r = w.size
    thr = threshold / fs if per_second else threshold
    idx = np.nonzero(np.abs(w) >= thr)[0]
    if idx.size == 0:
        return 0, np.zeros(0)
    signed = np.where(idx > n_r // 2, idx - n_r, idx)
    m_lo, m_hi = int(signed.min()), int(signed.max())
    return m_lo, w[np.arange(m_lo, m_hi + 1) % n_r].copy()


def reconstruct_bruteforce(z_ref: np.ndarray, m_lo: int, taps: np.ndarray, scale: float):
    """scale * sum_l z_ref[(m + m_lo + l) mod n] taps[l], term by term."""
    n = z_ref.size
    out = np.zeros(n, dtype=np.complex128)
    for l in range(taps.size):
        out += taps[l] * np.roll(z_ref, -(m_lo + l))
    return scale * out


def reconstruct(z_ref: np.ndarray, m_lo: int, taps: np.ndarray, scale: float):
    """Same circular correlation through a library FFT (exact up to rounding)."""
    n = z_ref.size
    if taps.size == 0:
        return np.zeros(n, dtype=np.complex128)
    if taps.size > n:
        raise ValueError("kernel longer than the segment")
    wfull = np.zeros(n, dtype=np.float64)
    np.add.at(wfull, (m_lo + np.arange(taps.size)) % n, taps)
    return scale * np.fft.ifft(np.fft.fft(z_ref) * np.conj(np.fft.fft(wfull)))


def reconstruct_oa(z_ref: np.ndarray, m_lo: int, taps: np.ndarray, scale: float):
    """Same circular correlation by overlap-add convolution (SciPy's
    oaconvolve, the routine the paper's CPU code uses, sec. IV): the series
    extended circularly by the kernel's span, convolved with the reversed
    taps, 'valid' part."""
    from scipy.signal import oaconvolve
    n = z_ref.size
    if taps.size == 0:
        return np.zeros(n, dtype=np.complex128)
    ext = z_ref[(m_lo + np.arange(n + taps.size - 1)) % n]
    return scale * oaconvolve(ext, taps[::-1], mode="valid")


def reconstruct_samples(z_ref, m_lo, taps, scale, sample_idx):
    """The defining sum evaluated only at the given output indices."""
    n = z_ref.size
    sample_idx = np.asarray(sample_idx, dtype=np.int64)
    cols = (sample_idx[:, None] + m_lo + np.arange(taps.size)[None, :]) % n
    return scale * (z_ref[cols] @ taps)


def analytic_window(f_low, f_high, df_lo, df_hi, ref, tgt, threshold):
    """Appendix-A time window outside which |r(t)| < threshold [s].

    Outside the chirp interval between dt(f_low) and dt(f_high) the tails are
    bounded by |R| / (4 pi df^2 |t - dt(f_edge)|^3) (equations flow_result_amp
    and fhigh_result_amp); setting the bound equal to the threshold gives a
    half-width t* = (|R| / (4 pi df^2 thr))^(1/3) about each edge.
    """
    r_amp = (taylorf2.mass_params(*tgt)[2] / taylorf2.mass_params(*ref)[2]) ** (5.0 / 6.0)
    dt_lo = float(taylorf2.time_of_frequency(f_low, *tgt) - taylorf2.time_of_frequency(f_low, *ref))
    dt_hi = float(taylorf2.time_of_frequency(f_high, *tgt) - taylorf2.time_of_frequency(f_high, *ref))
    ts_lo = (r_amp / (4.0 * math.pi * df_lo ** 2 * threshold)) ** (1.0 / 3.0)
    ts_hi = (r_amp / (4.0 * math.pi * df_hi ** 2 * threshold)) ** (1.0 / 3.0)
    return (min(dt_lo - ts_lo, dt_hi - ts_hi), max(dt_lo + ts_lo, dt_hi + ts_hi))


def interior_envelope(t, f_low, f_high, ref, tgt):
    """Appendix-A stationary-phase amplitude 2 |R| / sqrt(|dt'(f_dt(t))|) inside
    the chirp interval (equation delta_t_result; the modulus of its complex
    prefactor sqrt(2)(1 - i sgn) is 2).  f_dt(t) is found by bisection, which
    assumes dt(f) monotonic on the band as the appendix does.
    """
    r_amp = (taylorf2.mass_params(*tgt)[2] / taylorf2.mass_params(*ref)[2]) ** (5.0 / 6.0)

    def dt(f):
        return float(taylorf2.time_of_frequency(f, *tgt) - taylorf2.time_of_frequency(f, *ref))

    a, b = f_low, f_high
    ga, gb = dt(a) - t, dt(b) - t
    if ga * gb > 0:
        return None
    for _ in range(200):
        c = 0.5 * (a + b)
        gc = dt(c) - t
        if ga * gc <= 0:
            b, gb = c, gc
        else:
            a, ga = c, gc
    fc = 0.5 * (a + b)
    d2 = float(taylorf2.dtime_dfrequency(fc, *tgt) - taylorf2.dtime_dfrequency(fc, *ref))
    return 2.0 * r_amp / math.sqrt(abs(d2))


def build_kernel(grid, ref, tgt, threshold=1e-3, per_second=True, n_r=None):
    """Section II.C-II.D kernel for one (reference, target) pair on a grid-like object.

    Returns dict(m_lo, taps, df_low, norm_ratio) where norm_ratio = N_ref / N_k
    is left to the caller (it needs the PSD); here it is None.
    """
    n_r = grid.n if n_r is None else n_r
    dfl = df_low(grid.f_low, ref, tgt, grid.df_low_max)
    w = ratio_taps(grid.fs, n_r, grid.f_low, grid.f_high, dfl, grid.df_high, ref, tgt)
    m_lo, taps = truncate(w, grid.fs, threshold, per_second)
    return dict(m_lo=m_lo, taps=taps, df_low=dfl, full=w)


def project_kernel_set(kernels, rank: int):
    """Best rank-`rank` approximation of a set of truncated kernels.

    Not in the paper: the factored form of the reconstruction replaces every
    kernel of a set by its projection on the set's leading singular subspace
    (Eckart-Young: the rank-J matrix nearest the set in the Frobenius norm),
    then correlates as in section II.B eq. `convolution` with those kernels.
    kernels: list of (m_lo, taps).  The kernels are laid out on their union
    support [M0, M0 + L); the projection is taken from numpy's SVD of that
    K x L matrix.  Returns (M0, projected [K][L], relative residuals
    ||w_k - w~_k|| / ||w_k||).
    """
    live = [(m, t) for m, t in kernels if len(t)]
    m0 = min(m for m, _ in live)
    m1 = max(m + len(t) for m, t in live)
    W = np.zeros((len(kernels), m1 - m0))
    for k, (m, t) in enumerate(kernels):
        W[k, m - m0:m - m0 + len(t)] = t
    U, s, Vt = np.linalg.svd(W, full_matrices=False)
    J = min(rank, len(s))
    Wt = (U[:, :J] * s[:J]) @ Vt[:J]
    nrm = np.linalg.norm(W, axis=1)
    resid = np.linalg.norm(W - Wt, axis=1) / np.where(nrm > 0, nrm, 1.0)
    return m0, Wt, resid
