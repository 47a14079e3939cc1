"""Template-bank organisation (sec. III.A): the oracle against hand-worked
cases and invariants, and the library's host implementation against the
oracle on a synthetic stochastic bank (integer output: exact)."""
import numpy as np
import pytest

from oracle import bank as obank
from oracle import taylorf2 as otf2
from paper_2511_12894_amd import synth


def _equal_mass_bank(n):
    # chirp mass increases with the index
    return [(1.0 + 0.01 * i, 1.0 + 0.01 * i) for i in range(n)]


def test_oracle_chirp_mass_bisection_by_hand():
    """Durations 100, 99, 98, 97 | 80, 79 | 60, 59 (chirp-mass order): the whole
    bank spreads 41 s, its first half 3 s, its second half 21 s, whose halves
    spread 1 s each."""
    bank = _equal_mass_bank(8)
    tau = np.array([100.0, 99.0, 98.0, 97.0, 80.0, 79.0, 60.0, 59.0])
    groups, refs = obank.organise(bank, tau, max_spread=10.0, max_size=500)
    assert groups == [[0, 1, 2, 3], [4, 5], [6, 7]]
    # lower median duration: 98 (cost 1 + 1 + 2 = 4, as for 99), 79, 59
    assert refs == [2, 5, 7]


def test_oracle_eta_bisection_and_odd_halves():
    """One duration set of 5 templates split along symmetric mass ratio to at
    most 2: halves of 5 are 2 + 3, the 3 becomes 1 + 2."""
    bank = [(1.5, 1.5), (2.0, 1.1), (1.6, 1.4), (2.4, 1.0), (1.8, 1.25)]
    eta = [m1 * m2 / (m1 + m2) ** 2 for m1, m2 in bank]
    tau = np.full(5, 50.0)
    groups, refs = obank.organise(bank, tau, max_spread=10.0, max_size=2)
    by_eta = sorted(range(5), key=lambda i: eta[i])
    assert groups == [by_eta[:2], by_eta[2:3], by_eta[3:]]
    # equal durations: the first template of each set
    assert refs == [by_eta[0], by_eta[2], by_eta[3]]


def test_oracle_reference_minimises_summed_difference():
    rng = np.random.default_rng(3)
    for size in (1, 2, 3, 7, 10):
        tau = rng.uniform(0, 10, size)
        bank = _equal_mass_bank(size)
        groups, refs = obank.organise(bank, tau, max_spread=100.0, max_size=500)
        assert len(groups) == 1
        cost = [np.abs(tau - tau[i]).sum() for i in range(size)]
        r = refs[0]
        assert cost[r] <= min(cost) * (1 + 1e-12)
        # a median: at least half the durations on either side
        assert np.sum(tau <= tau[r]) >= size / 2 and np.sum(tau >= tau[r]) >= size / 2


@pytest.fixture(scope="module")
def sbank():
    """Synthetic stochastic bank over 1-1.6 Msun at f_low = 20 Hz."""
    b = synth.stochastic_bank(m_range=(1.0, 1.6))
    return b, obank.durations(b, 20.0)


def test_oracle_invariants_on_a_stochastic_bank(sbank):
    b, tau = sbank
    assert len(b) > 1000
    groups, refs = obank.organise(b, tau, max_spread=10.0, max_size=500)
    flat = sorted(i for g in groups for i in g)
    assert flat == list(range(len(b)))
    for g, r in zip(groups, refs):
        assert len(g) <= 500 and r in g
        tg = tau[g]
        assert tg.max() - tg.min() <= 10.0
    # the duration bisection is as coarse as the rule allows: merging the two
    # halves of any split would break the 10 s spread or the size limit
    assert len(groups) >= 2


def test_durations_match_the_oracle(sbank):
    from paper_2511_12894_amd import rf
    b, tau = sbank
    tl = rf.template_durations(b, 20.0)
    assert np.abs(tl - tau).max() <= 1e-12 * tau.max()
    # Newtonian limit of a light, equal-mass system: tau ~ tau0 (leading order)
    t0, _ = synth.chirp_times(1.0, 1.0, 20.0)
    assert abs(float(otf2.duration(np.array([20.0]), 1.0, 1.0)[0]) / t0 - 1.0) < 0.05


@pytest.mark.parametrize("spread,size", [(10.0, 500), (10.0, 100), (2.0, 37), (0.0, 500), (1e9, 1)])
def test_library_matches_the_oracle(sbank, spread, size):
    from paper_2511_12894_amd import rf
    b, tau = sbank
    if spread == 0.0:
        b, tau = b[:300], tau[:300]
    groups, refs = obank.organise(b, tau, max_spread=spread, max_size=size)
    g_lib, r_lib = rf.bank_organise(b, tau, max_spread=spread, max_size=size)
    exp = np.empty(len(b), dtype=np.int32)
    for gi, g in enumerate(groups):
        exp[g] = gi
    assert np.array_equal(g_lib, exp)
    assert list(r_lib) == list(refs)


def test_library_edge_cases_and_errors():
    from paper_2511_12894_amd import rf
    g, r = rf.bank_organise([(1.4, 1.4)], [10.0])
    assert list(g) == [0] and list(r) == [0]
    b = _equal_mass_bank(6)
    g, r = rf.bank_organise(b, np.full(6, 3.0), max_spread=0.0, max_size=4)
    assert list(g) == [0, 0, 0, 1, 1, 1] and list(r) == [0, 3]
    for args in ((b, np.full(6, np.nan)), ([], [])):
        with pytest.raises(rf.RfError) as e:
            rf.bank_organise(*args)
        assert e.value.code == rf.RF_E_INVAL
    with pytest.raises(rf.RfError):
        rf.bank_organise(b, np.zeros(6), max_size=0)
