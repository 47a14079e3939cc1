"""Seeded synthetic inputs for the ratio-filter hot path.

This module makes the data that both the HIP library and the FP64 oracle are
fed: a one-sided PSD, coloured Gaussian noise in the frequency domain, signal
injections and template parameter sets.  It holds none of the filtering
arithmetic (no matched filter, no ratio kernel, no reconstruction, no peak
search).  The injected signals need a waveform; it is this module's own
writing of the non-spinning TaylorF2 source model (stationary-phase form of
the paper's appendix A, 3.5PN phase, Newtonian amplitude), used only to
simulate the detector data.

Conventions (paper section II): a~(f) = int a(t) exp(-2 pi i f t) dt, and a
frequency series is stored for bins j = 0..n/2 at f_j = j * fs / n.

The paper's mock data (section III.B) use the tabulated zero-detuned
high-power advanced-detector PSD, which is not available here; the analytic
fit of that curve (Ajith 2011 form, f0 = 215 Hz) stands in for it.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# G M_sun / c^3 in seconds (IAU 2015 nominal solar mass parameter).
T_SUN_S = 4.925490947641267e-6
_EULER_GAMMA = 0.5772156649015329


@dataclasses.dataclass(frozen=True)
class Grid:
    """Sampling of one data segment and the analysis band.

    fs: sample rate [Hz]; n: samples (a power of two); f_low, f_high: band
    edges [Hz] (section II.A); df_high: upper taper width (53 Hz, section
    II.C); df_low_max: cap on the lower taper width (5 Hz, section II.C).
    """

    fs: float
    n: int
    f_low: float
    f_high: float
    df_high: float = 53.0
    df_low_max: float = 5.0

    @property
    def duration(self) -> float:
        return self.n / self.fs

    @property
    def df(self) -> float:
        return self.fs / self.n

    def freqs(self) -> np.ndarray:
        return np.arange(self.n // 2 + 1, dtype=np.float64) * self.df


def make_grid(fs: float, n: int, f_low: float, df_high: float = 53.0,
              df_low_max: float = 5.0) -> Grid:
    """Grid whose upper taper ends exactly at Nyquist: f_high = fs/2 - df_high.

    The paper keeps f_high = 2048 Hz at fs = 4096 Hz and zero-pads the spectrum
    to 2101 Hz (section IV); placing f_high one taper width below Nyquist keeps
    the whole window of equation (window) inside the sampled band instead.
    """
    return Grid(float(fs), int(n), float(f_low), float(fs) / 2.0 - df_high,
                df_high, df_low_max)


# ---------------------------------------------------------------- noise model

def psd_fit(f: np.ndarray) -> np.ndarray:
    """Analytic fit of the zero-detuned high-power design PSD [1/Hz].

    S(f) = 1e-49 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2) / (1 + x^2/2)],
    x = f / 215 Hz.  Bin 0 (x = 0) is given the value of bin 1; it lies
    outside every analysis band.
    """
    f = np.asarray(f, dtype=np.float64)
    x = np.where(f > 0, f, 1.0) / 215.0
    s = 1e-49 * (x ** -4.14 - 5.0 * x ** -2
                 + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))
    if s.ndim and f[0] == 0.0 and s.size > 1:
        s[0] = s[1]
    return s


def make_psd(grid: Grid) -> np.ndarray:
    return psd_fit(grid.freqs())


def noise(grid: Grid, psd: np.ndarray, seed: int) -> np.ndarray:
    """Stationary coloured Gaussian noise x~_j, j = 0..n/2 (complex128).

    Each positive-frequency bin is sqrt(T S_j / 4) (a + i b) with a, b
    independent N(0, 1), so that E|x~_j|^2 = T S_j / 2 for the one-sided PSD
    S.  DC is zero and the Nyquist bin is real.
    """
    rng = np.random.default_rng(seed)
    m = grid.n // 2 + 1
    a = rng.standard_normal(m)
    b = rng.standard_normal(m)
    scale = np.sqrt(grid.duration * psd / 4.0)
    x = scale * (a + 1j * b)
    x[0] = 0.0
    x[-1] = np.sqrt(grid.duration * psd[-1] / 2.0) * a[-1]
    return x


# --------------------------------------------------------- source (injection)

def _source_phase(f: np.ndarray, m1: float, m2: float) -> np.ndarray:
    """TaylorF2 stationary-phase phase with t_c = phi_c = 0 [rad].

    Psi(f) = -pi/4 + 3/(128 eta) sum_k a_k v^(k-5), v = (pi M f)^(1/3); the
    coefficients a_k are the published non-spinning 3.5PN values written out
    as rationals in eta.
    """
    mt = (m1 + m2) * T_SUN_S
    eta = m1 * m2 / (m1 + m2) ** 2
    v = np.cbrt(math.pi * mt * f)
    lv = np.log(v)
    pi = math.pi
    a0 = 1.0
    a2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta
    a3 = -16.0 * pi
    a4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta ** 2
    a5 = pi * (38645.0 / 756.0 - 65.0 / 9.0 * eta) * (1.0 + 3.0 * (lv + 0.5 * math.log(6.0)))
    a6 = (11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi ** 2
          - 6848.0 / 21.0 * _EULER_GAMMA - 6848.0 / 21.0 * (math.log(4.0) + lv)
          + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi ** 2) * eta
          + 76055.0 / 1728.0 * eta ** 2 - 127825.0 / 1296.0 * eta ** 3)
    a7 = pi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta
               - 74045.0 / 756.0 * eta ** 2)
    poly = a0 + v * v * (a2 + v * (a3 + v * (a4 + v * (a5 + v * (a6 + v * a7)))))
    return -0.25 * pi + 3.0 / (128.0 * eta) * poly / v ** 5


def source_spectrum(grid: Grid, m1: float, m2: float, t0: float, phi0: float,
                    f_min: float) -> np.ndarray:
    """Unit-scaled source signal e^{i phi0} B(f) e^{-i Psi(f)} e^{-2 pi i f t0}.

    B(f) = Mc^(5/6) f^(-7/6) (Mc in seconds; overall constants dropped).
    Non-zero for f_min <= f < fs/2.
    """
    f = grid.freqs()
    sel = (f >= f_min) & (f < grid.fs / 2.0)
    out = np.zeros(f.shape, dtype=np.complex128)
    fs_ = f[sel]
    mt = (m1 + m2) * T_SUN_S
    mc = mt * (m1 * m2 / (m1 + m2) ** 2) ** 0.6
    amp = mc ** (5.0 / 6.0) * fs_ ** (-7.0 / 6.0)
    ph = -_source_phase(fs_, m1, m2) - 2.0 * math.pi * fs_ * t0 + phi0
    out[sel] = amp * np.exp(1j * ph)
    return out


def inject(grid: Grid, psd: np.ndarray, xf: np.ndarray, m1: float, m2: float,
           snr: float, t0: float, phi0: float) -> np.ndarray:
    """Add a source whose optimal SNR over [f_low, f_high] is `snr`.

    Optimal SNR^2 = 4 df sum_band |s_j|^2 / S_j (section II.A with the band
    limit); the source is scaled to meet it.  Returns a new array.
    """
    s = source_spectrum(grid, m1, m2, t0, phi0, grid.f_low - grid.df_low_max)
    f = grid.freqs()
    band = (f >= grid.f_low) & (f <= grid.f_high)
    rho2 = 4.0 * grid.df * np.sum(np.abs(s[band]) ** 2 / psd[band])
    return xf + (snr / math.sqrt(rho2)) * s


# ------------------------------------------------------ template parameters

def chirp_times(m1: float, m2: float, f0: float) -> tuple[float, float]:
    """Newtonian and 1.5PN chirp times (tau0, tau3) at f0 [s]."""
    mt = (m1 + m2) * T_SUN_S
    eta = m1 * m2 / (m1 + m2) ** 2
    x = math.pi * mt * f0
    tau0 = 5.0 / (256.0 * math.pi * f0 * eta) * x ** (-5.0 / 3.0)
    tau3 = 1.0 / (8.0 * f0 * eta) * x ** (-2.0 / 3.0)
    return tau0, tau3


def masses_from_chirp_times(tau0: float, tau3: float, f0: float):
    """Inverse of chirp_times; None when the point is unphysical (eta > 1/4)."""
    mt = 5.0 * tau3 / (32.0 * math.pi ** 2 * f0 * tau0)
    eta = (math.pi * mt * f0) ** (-2.0 / 3.0) / (8.0 * f0 * tau3)
    if not (0.0 < eta <= 0.25) or mt <= 0.0:
        return None
    m = mt / T_SUN_S
    d = math.sqrt(max(0.0, 1.0 - 4.0 * eta))
    return 0.5 * m * (1.0 + d), 0.5 * m * (1.0 - d)


# Lattice steps of the stand-in for a minimal-match-0.97 placement: relative
# steps in chirp mass and symmetric mass ratio, mapped to chirp times
# (dtau0/tau0 = -5/3 dMc/Mc, dtau3/tau3 = -3/5 deta/eta at fixed Mc).
_DMC_REL = 1.33e-4
_DETA_REL = 1.31e-2


def neighbour_lattice(m1: float, m2: float, f0: float, count: int):
    """`count` lattice points nearest a reference in (tau0, tau3).

    The lattice has steps (5/3 * 1.33e-4 tau0_ref, 3/5 * 1.31e-2 tau3_ref),
    excludes the reference itself and unphysical points, and is ordered by
    lattice distance (ties by index).  Returns a list of (m1, m2).
    """
    t0r, t3r = chirp_times(m1, m2, f0)
    d0 = 5.0 / 3.0 * _DMC_REL * t0r
    d3 = 3.0 / 5.0 * _DETA_REL * t3r
    radius = 4
    while True:
        pts = []
        for i in range(-radius, radius + 1):
            for j in range(-radius, radius + 1):
                if i == 0 and j == 0:
                    continue
                ms = masses_from_chirp_times(t0r + i * d0, t3r + j * d3, f0)
                if ms is not None:
                    pts.append((i * i + j * j, i, j, ms))
        pts.sort(key=lambda p: (p[0], p[1], p[2]))
        if len(pts) >= count and pts[count - 1][0] < radius * radius:
            return [p[3] for p in pts[:count]]
        radius *= 2


def stochastic_bank(f0: float = 20.0, m_range=(1.0, 3.0), seed: int = 1006, fiducial=(1.6, 1.2),
                    sub: int = 4):
    """Stand-in for a minimal-match-0.97 stochastic placement over m1, m2 in
    `m_range`: candidates on a jittered grid of 1/`sub` lattice step in
    (tau0, tau3), visited in seeded random order, are accepted when no
    accepted point lies within one lattice step (the steps of
    `neighbour_lattice` at the fiducial masses, taken as constant: the metric
    is nearly flat in chirp times).  Returns a list of (m1, m2), m1 >= m2, in
    acceptance order."""
    lo_m, hi_m = m_range
    t0f, t3f = chirp_times(*fiducial, f0)
    d0 = 5.0 / 3.0 * _DMC_REL * t0f
    d3 = 3.0 / 5.0 * _DETA_REL * t3f
    corners = [chirp_times(a, b, f0) for a in (lo_m, hi_m) for b in (lo_m, hi_m)]
    u0, u1 = min(c[0] for c in corners) / d0, max(c[0] for c in corners) / d0
    v0, v1 = min(c[1] for c in corners) / d3, max(c[1] for c in corners) / d3
    rng = np.random.default_rng(seed)
    uu, vv = np.meshgrid(np.arange(u0, u1, 1.0 / sub), np.arange(v0, v1, 1.0 / sub), indexing="ij")
    cand = np.column_stack([uu.ravel(), vv.ravel()]) + rng.uniform(0.0, 1.0 / sub, (uu.size, 2))
    cand = cand[rng.permutation(len(cand))]
    # the physical part of the mass range (vectorised masses_from_chirp_times)
    t0, t3 = cand[:, 0] * d0, cand[:, 1] * d3
    mt = 5.0 * t3 / (32.0 * math.pi ** 2 * f0 * t0)
    with np.errstate(invalid="ignore", divide="ignore"):
        eta = (math.pi * mt * f0) ** (-2.0 / 3.0) / (8.0 * f0 * t3)
        dd = np.sqrt(np.maximum(0.0, 1.0 - 4.0 * eta))
    m = mt / T_SUN_S
    m1, m2 = 0.5 * m * (1.0 + dd), 0.5 * m * (1.0 - dd)
    keep = (eta > 0.0) & (eta <= 0.25) & (mt > 0.0) & (m2 >= lo_m) & (m1 <= hi_m)
    cells = {}
    bank = []
    for u, v, a, b in zip(cand[keep, 0].tolist(), cand[keep, 1].tolist(), m1[keep].tolist(), m2[keep].tolist()):
        ms = (a, b)
        cu, cv = int(math.floor(u)), int(math.floor(v))
        near = False
        for du in (-1, 0, 1):
            for dv in (-1, 0, 1):
                for (pu, pv) in cells.get((cu + du, cv + dv), ()):
                    if (pu - u) ** 2 + (pv - v) ** 2 < 1.0:
                        near = True
                        break
                if near:
                    break
            if near:
                break
        if near:
            continue
        cells.setdefault((cu, cv), []).append((u, v))
        bank.append(ms)
    return bank


def masses_from_mc_q(mc: float, q: float):
    """(m1, m2), m1 >= m2, of chirp mass `mc` and mass ratio q = m2 / m1."""
    m1 = mc * (1.0 + q) ** 0.2 * q ** -0.6
    return m1, q * m1


# ------------------------------------------------------------------ workloads

def workload_small():
    """Plain method, small case: 64 s at 1024 Hz, f_low = 30 Hz.

    Reference 1.4+1.4; 16 equal-mass neighbours with chirp mass scaled by
    1 +- {0.05, 0.10, ..., 0.40} %; one 1.4+1.4 injection at SNR 12, t0 = 40 s.
    """
    grid = make_grid(1024.0, 65536, 30.0)
    psd = make_psd(grid)
    xf = noise(grid, psd, seed=1001)
    xf = inject(grid, psd, xf, 1.4, 1.4, 12.0, 40.0, 0.0)
    ref = (1.4, 1.4)
    nbrs = []
    for pct in np.arange(1, 9) * 0.05:
        for sgn in (-1.0, 1.0):
            m = 1.4 * (1.0 + sgn * pct / 100.0)
            nbrs.append((m, m))
    return dict(name="small-64s-1024Hz-1ref-16nbr", grid=grid, psd=psd, xf=xf,
                ref=ref, nbrs=nbrs, injections=[(1.4, 1.4, 12.0, 40.0, 0.0)])


def workload_realistic(n_nbr: int = 256, seed: int = 1002, duration: float = 512.0,
                       fs: float = 4096.0):
    """Single reference, realistic: 512 s at 4096 Hz, f_low = 20 Hz.

    Reference 1.6+1.2 with `n_nbr` lattice neighbours; four injections at
    SNR 8, 12, 16, 20 at t0 = 100, 200, 300, 400 s with masses of four seeded
    neighbours and uniform random phases.  `duration`/`fs` may be reduced for
    test-sized variants of the same structure.
    """
    n = int(round(duration * fs))
    grid = make_grid(fs, n, 20.0)
    psd = make_psd(grid)
    xf = noise(grid, psd, seed=seed)
    ref = (1.6, 1.2)
    nbrs = neighbour_lattice(ref[0], ref[1], grid.f_low, n_nbr)
    rng = np.random.default_rng(seed + 1000)
    pick = rng.choice(len(nbrs), size=4, replace=False)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=4)
    injections = []
    for i, (snr, t0) in enumerate(zip((8.0, 12.0, 16.0, 20.0), (100.0, 200.0, 300.0, 400.0))):
        t0 = t0 * duration / 512.0
        m1, m2 = nbrs[int(pick[i])]
        xf = inject(grid, psd, xf, m1, m2, snr, t0, float(phases[i]))
        injections.append((m1, m2, snr, t0, float(phases[i])))
    return dict(name=f"realistic-{duration:g}s-{fs:g}Hz-1ref-{n_nbr}nbr", grid=grid,
                psd=psd, xf=xf, ref=ref, nbrs=nbrs, injections=injections)


def workload_batched(n_seg: int = 8, n_ref: int = 64, duration: float = 256.0,
                     fs: float = 4096.0, f_low: float = 25.0, seed: int = 1003,
                     nbr_range=(32, 512)):
    """Batched uneven: `n_seg` segments, `n_ref` references with m1, m2 ~ U[1, 3].

    Each reference gets floor(exp U[ln lo, ln hi]) lattice neighbours.  One
    injection per segment at SNR 10, masses of a seeded neighbour.
    """
    n = int(round(duration * fs))
    grid = make_grid(fs, n, f_low)
    psd = make_psd(grid)
    rng = np.random.default_rng(seed)
    refs, groups = [], []
    for _ in range(n_ref):
        a, b = rng.uniform(1.0, 3.0, size=2)
        m1, m2 = max(a, b), min(a, b)
        k = int(math.floor(math.exp(rng.uniform(math.log(nbr_range[0]), math.log(nbr_range[1])))))
        refs.append((float(m1), float(m2)))
        groups.append(neighbour_lattice(m1, m2, f_low, k))
    segs, injections = [], []
    for s in range(n_seg):
        xf = noise(grid, psd, seed=seed + 10 * (s + 1))
        g = int(rng.integers(n_ref))
        m1, m2 = groups[g][int(rng.integers(len(groups[g])))]
        t0 = float(rng.uniform(0.2, 0.8) * duration)
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
        xf = inject(grid, psd, xf, m1, m2, 10.0, t0, phi)
        segs.append(xf)
        injections.append((s, m1, m2, 10.0, t0, phi))
    return dict(name=f"batched-{n_seg}seg-{duration:g}s-{n_ref}ref", grid=grid, psd=psd,
                segments=segs, refs=refs, groups=groups, injections=injections)


def workload_stress(n_nbr: int = 1024, refs=((1.0, 1.0), (1.167, 1.167), (1.333, 1.333), (1.5, 1.5)),
                    duration: float = 2048.0, fs: float = 4096.0, f_low: float = 10.0, seed: int = 1005):
    """Next-generation-detector shape: 2048 s at 4096 Hz (n = 2^23), f_low = 10 Hz,
    equal-mass references with `n_nbr` lattice neighbours each, one injection at
    SNR 15 at t0 = 1000 s on a seeded neighbour of the first reference."""
    n = int(round(duration * fs))
    grid = make_grid(fs, n, f_low)
    psd = make_psd(grid)
    rng = np.random.default_rng(seed)
    groups = [neighbour_lattice(m1, m2, f_low, n_nbr) for m1, m2 in refs]
    xf = noise(grid, psd, seed=seed)
    m1, m2 = groups[0][int(rng.integers(n_nbr))]
    phi = float(rng.uniform(0.0, 2.0 * math.pi))
    xf = inject(grid, psd, xf, m1, m2, 15.0, 1000.0, phi)
    return dict(name=f"stress-{duration:g}s-{fs:g}Hz-{len(refs)}ref-{n_nbr}nbr", grid=grid, psd=psd, xf=xf,
                refs=[tuple(r) for r in refs], groups=groups, injections=[(m1, m2, 15.0, 1000.0, phi)])


# ------------------------------------------------------- learned-kernel inputs

def surrogate_pairs(f0: float, count: int, seed: int, m_range=(1.0, 3.0), steps: int = 10):
    """Training pairs: references with m1, m2 ~ U[m_range] (m1 >= m2) and a
    neighbour at a random offset of at most `steps` lattice steps in each
    chirp-time direction (the lattice of neighbour_lattice)."""
    rng = np.random.default_rng(seed)
    refs, nbrs = [], []
    while len(refs) < count:
        a, b = rng.uniform(*m_range, size=2)
        ref = (float(max(a, b)), float(min(a, b)))
        t0r, t3r = chirp_times(*ref, f0)
        i, j = rng.integers(-steps, steps + 1, size=2)
        ms = masses_from_chirp_times(t0r + i * 5.0 / 3.0 * _DMC_REL * t0r, t3r + j * 3.0 / 5.0 * _DETA_REL * t3r, f0)
        if ms is None:
            continue
        refs.append(ref)
        nbrs.append(ms)
    return refs, nbrs


def surrogate_random_inputs(seed: int, npair: int, nomega: int, steps: int, batch: int):
    """Random numbers the surrogate's construction and training draw: standard
    normal range-finder draws [npair][nomega], initial parameters (weights
    N(0, 2/fan_in), zero biases, packed W1 b1 W2 b2 W3 b3 W4 b4) and the batch
    order (shuffled epochs) [steps][batch]."""
    rng = np.random.default_rng(seed)
    omega = rng.standard_normal((npair, nomega))
    parts = []
    for fi, fo in ((4, 256), (256, 256), (256, 256), (256, 128)):
        parts.append((rng.standard_normal((fo, fi)) * np.sqrt(2.0 / fi)).ravel())
        parts.append(np.zeros(fo))
    theta = np.concatenate(parts).astype(np.float32)
    need = steps * batch
    order = np.concatenate([rng.permutation(npair) for _ in range(need // npair + 1)])[:need]
    return omega, theta, order.reshape(steps, batch).astype(np.int32)


def workload_sweep(mc: float, q: float, snr: float = 20.0, seed: int = 1007, duration: float = 512.0,
                   fs: float = 4096.0, f_low: float = 20.0, t0: float = 400.0):
    """Accuracy sweep case (the paper's SNR-loss study): 512 s at 4096 Hz,
    f_low = 20 Hz, coloured noise plus one injection of chirp mass `mc` and
    mass ratio q at optimal SNR `snr`, coalescing at t0; the reference of the
    study has the same chirp mass and q = 0.6."""
    n = int(round(duration * fs))
    grid = make_grid(fs, n, f_low)
    psd = make_psd(grid)
    tgt = masses_from_mc_q(mc, q)
    xf = noise(grid, psd, seed=seed + int(round(1000 * q)))
    xf = inject(grid, psd, xf, tgt[0], tgt[1], snr, t0, 0.0)
    return dict(name=f"sweep-mc{mc}-q{q}", grid=grid, psd=psd, xf=xf, ref=masses_from_mc_q(mc, 0.6), tgt=tgt,
                t0=t0)
