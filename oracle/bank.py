"""Template-bank organisation into reference / dependent sets (sec. III.A,
template bank construction), written from the paper's description.

Test infrastructure only: imported by tests/, the smoke check and bench.py's
CPU baseline, never by the product path.

Steps, in the paper's order:
  1. Order the bank by chirp mass and split it into two halves, again and
     again, until in every subset the longest and shortest waveform durations
     differ by at most `max_spread` (10 s in the paper).
  2. Split every subset with more than `max_size` templates (500 in the paper)
     into halves along symmetric mass ratio, again and again, until none is
     larger.
  3. In every set, the reference is the template minimising the summed
     absolute duration difference to all templates of the set.
Durations are tau(f_low) from the TaylorF2 phase (sec. II.C).

Readings (the paper does not fix them): "halves" of an odd count put the
smaller half first; ties in chirp mass or symmetric mass ratio keep the
previous order (stable sorts, starting from bank index); among templates that
minimise the summed difference (two, for an even count of distinct
durations) the one with the shorter duration is taken.
"""
import numpy as np

from . import taylorf2


def durations(bank, f_low: float) -> np.ndarray:
    """tau(f_low) of each (m1, m2) of the bank."""
    return np.array([float(taylorf2.duration(np.array([f_low]), m1, m2)[0]) for m1, m2 in bank])


def chirp_mass_and_eta(m1: float, m2: float):
    m = m1 + m2
    eta = m1 * m2 / (m * m)
    return m * eta ** 0.6, eta


def _halves(items, ok):
    """Split the list `items` in halves until ok(part) holds for every part."""
    if len(items) <= 1 or ok(items):
        return [items]
    mid = len(items) // 2
    return _halves(items[:mid], ok) + _halves(items[mid:], ok)


def organise(bank, tau, max_spread: float = 10.0, max_size: int = 500):
    """Returns (groups, references): groups as lists of bank indices in the
    order the procedure visits them, references[g] the index of group g's
    reference template."""
    mc_eta = [chirp_mass_and_eta(m1, m2) for m1, m2 in bank]
    by_mc = sorted(range(len(bank)), key=lambda i: mc_eta[i][0])
    spread_ok = lambda part: max(tau[i] for i in part) - min(tau[i] for i in part) <= max_spread
    sets = _halves(by_mc, spread_ok)
    groups = []
    for s in sets:
        by_eta = sorted(s, key=lambda i: mc_eta[i][1])
        groups += _halves(by_eta, lambda part: len(part) <= max_size)
    refs = []
    for g in groups:
        tg = np.array([tau[i] for i in g])
        cost = np.abs(tg[:, None] - tg[None, :]).sum(axis=1)
        best = cost.min()
        # the minimisers (equal up to rounding of the sums): the shortest
        # duration, then the first in the set's order
        cands = [p for p in range(len(g)) if cost[p] <= best * (1 + 1e-12)]
        refs.append(g[min(cands, key=lambda p: (tg[p], p))])
    return groups, refs
