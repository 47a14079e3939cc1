"""Oracle: peak and threshold read-out of SNR series (section IV compares the
peak |z| of the standard and ratio-filter series).

For each series: rho_max = max_m |z[m]| with the smallest index on ties; a
trigger is every (template, m) with |z[m]| strictly above the threshold,
listed in (template, m) order.
"""
from __future__ import annotations

import numpy as np


def peak(z: np.ndarray):
    a = np.abs(z)
    i = int(np.argmax(a))          # numpy returns the first maximum
    return float(a[i]), i


def triggers(z_rows, threshold: float):
    """List of (template, index, |z|, arg z) with |z| > threshold."""
    out = []
    for k, z in enumerate(z_rows):
        a = np.abs(z)
        for m in np.nonzero(a > threshold)[0]:
            out.append((k, int(m), float(a[m]), float(np.angle(z[m]))))
    return out


def peak_loop(z):
    """The same maximum by a plain Python loop (small inputs)."""
    best, arg = -1.0, -1
    for m, v in enumerate(z):
        a = abs(complex(v))
        if a > best:
            best, arg = a, m
    return best, arg
