"""Oracle: non-spinning TaylorF2 waveform in stationary-phase form.

The paper builds every template with the TaylorF2 model (section II.B, Fig. 1;
section III.B) and writes a frequency-domain waveform as h~(f) = B(f)
exp(-i Psi(f)) with Psi'(f) = 2 pi t(f) (appendix A).  The phase series is the
published non-spinning 3.5PN one (the paper's TaylorF2 citation, Buonanno et
al. 2009), with coalescence time and phase set to zero:

    Psi(f) = -pi/4 + 3 / (128 eta v^5) * sum_k psi_k v^k,   v = (pi M f)^(1/3)

and the amplitude is the Newtonian B(f) = Mc^(5/6) f^(-7/6) (overall constants
dropped: every SNR is normalised and every kernel is a ratio, so they cancel).
Masses are in solar masses and converted to seconds with G M_sun / c^3.
"""
from __future__ import annotations

import math

import numpy as np

T_SUN = 4.925490947641267e-6          # G M_sun / c^3 [s]
GAMMA_E = 0.5772156649015329          # Euler-Mascheroni constant
V_LSO = 1.0 / math.sqrt(6.0)          # velocity at the last stable orbit


def mass_params(m1: float, m2: float):
    """Total mass M [s], symmetric mass ratio eta, chirp mass Mc [s]."""
    mt = (m1 + m2) * T_SUN
    eta = m1 * m2 / (m1 + m2) ** 2
    return mt, eta, mt * eta ** 0.6


def phase_coefficients(eta: float) -> dict:
    """psi_k of the 3.5PN series (Buonanno et al. 2009 form).

    psi_5 multiplies (1 + 3 ln(v / v_lso)); psi_6 = c6 + c6l * ln(4 v).
    """
    pi = math.pi
    return dict(
        c0=1.0,
        c2=20.0 / 9.0 * (743.0 / 336.0 + 11.0 / 4.0 * eta),
        c3=-16.0 * pi,
        c4=10.0 * (3058673.0 / 1016064.0 + 5429.0 / 1008.0 * eta + 617.0 / 144.0 * eta ** 2),
        c5=pi * (38645.0 / 756.0 - 65.0 / 9.0 * eta),
        c6=(11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi ** 2
            - 6848.0 / 21.0 * GAMMA_E
            + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi ** 2) * eta
            + 76055.0 / 1728.0 * eta ** 2 - 127825.0 / 1296.0 * eta ** 3),
        c6l=-6848.0 / 21.0,
        c7=pi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta ** 2),
    )


def _series(v: np.ndarray, eta: float):
    """P(v) = 3/(128 eta) sum_k psi_k(v) v^(k-5) and its first two v-derivatives."""
    c = phase_coefficients(eta)
    lv = np.log(v)
    l5 = 1.0 + 3.0 * (lv - math.log(V_LSO))
    c6v = c["c6"] + c["c6l"] * (math.log(4.0) + lv)
    p = (c["c0"] * v ** -5 + c["c2"] * v ** -3 + c["c3"] * v ** -2 + c["c4"] / v
         + c["c5"] * l5 + c6v * v + c["c7"] * v ** 2)
    dp = (-5.0 * c["c0"] * v ** -6 - 3.0 * c["c2"] * v ** -4 - 2.0 * c["c3"] * v ** -3
          - c["c4"] * v ** -2 + 3.0 * c["c5"] / v + (c6v + c["c6l"]) + 2.0 * c["c7"] * v)
    d2p = (30.0 * c["c0"] * v ** -7 + 12.0 * c["c2"] * v ** -5 + 6.0 * c["c3"] * v ** -4
           + 2.0 * c["c4"] * v ** -3 - 3.0 * c["c5"] / v ** 2 + c["c6l"] / v + 2.0 * c["c7"])
    k = 3.0 / (128.0 * eta)
    return k * p, k * dp, k * d2p


def phase(f, m1: float, m2: float) -> np.ndarray:
    """Psi(f) [rad] with t_c = phi_c = 0 (appendix A's h~ = B e^{-i Psi})."""
    mt, eta, _ = mass_params(m1, m2)
    f = np.asarray(f, dtype=np.float64)
    v = np.cbrt(math.pi * mt * f)
    p, _, _ = _series(v, eta)
    return -0.25 * math.pi + p


def time_of_frequency(f, m1: float, m2: float) -> np.ndarray:
    """t(f) = Psi'(f) / (2 pi) [s] (appendix A); negative before coalescence."""
    mt, eta, _ = mass_params(m1, m2)
    f = np.asarray(f, dtype=np.float64)
    v = np.cbrt(math.pi * mt * f)
    _, dp, _ = _series(v, eta)
    dv = v / (3.0 * f)
    return dp * dv / (2.0 * math.pi)


def dtime_dfrequency(f, m1: float, m2: float) -> np.ndarray:
    """t'(f) = Psi''(f) / (2 pi) [s/Hz] (appendix A)."""
    mt, eta, _ = mass_params(m1, m2)
    f = np.asarray(f, dtype=np.float64)
    v = np.cbrt(math.pi * mt * f)
    _, dp, d2p = _series(v, eta)
    dv = v / (3.0 * f)
    d2v = -2.0 * v / (9.0 * f * f)
    return (d2p * dv * dv + dp * d2v) / (2.0 * math.pi)


def amplitude(f, m1: float, m2: float) -> np.ndarray:
    """Newtonian amplitude B(f) = Mc^(5/6) f^(-7/6) (constants dropped)."""
    _, _, mc = mass_params(m1, m2)
    f = np.asarray(f, dtype=np.float64)
    return mc ** (5.0 / 6.0) * f ** (-7.0 / 6.0)


def template(f, m1: float, m2: float) -> np.ndarray:
    """h~(f) = B(f) exp(-i Psi(f)); zero where f <= 0."""
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros(f.shape, dtype=np.complex128)
    pos = f > 0
    out[pos] = amplitude(f[pos], m1, m2) * np.exp(-1j * phase(f[pos], m1, m2))
    return out


def duration(f, m1: float, m2: float) -> np.ndarray:
    """tau(f): time from frequency f to merger, t_c - t(f) with t_c = 0 (section II.C)."""
    return -time_of_frequency(f, m1, m2)
