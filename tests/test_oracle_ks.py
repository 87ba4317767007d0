"""Pins of the oracle's KS distance (Sec. 3.1, eq. KS): the largest gap
between two empirical CDFs, bounded by one and unchanged by monotone maps of
the samples."""
import numpy as np
import pytest
from scipy.stats import ks_2samp


def test_ks_special_cases(orc):
    a = np.array([1.0, 2.0, 3.0])
    assert orc.ks_distance(a, a) == 0.0
    assert orc.ks_distance(a, a + 10.0) == 1.0
    # F - G at x = 2: 2/3 of a against none of b (b = {2.5})
    assert orc.ks_distance(a, [2.5]) == pytest.approx(2.0 / 3.0, abs=1e-15)
    # a tie across the samples: at x = 2 all of a = {1, 2, 2} and one of
    # b = {2, 3, 4, 5} lie at or below x, F - G = 1 - 1/4
    assert orc.ks_distance([1.0, 2.0, 2.0], [2.0, 3.0, 4.0, 5.0]) == pytest.approx(0.75, abs=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ks_matches_library_two_sample_statistic(orc, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(700)
    b = 0.3 + 1.2 * rng.standard_normal(450)
    b[:40] = a[:40]   # shared values (ties across the samples)
    want = ks_2samp(a, b).statistic
    assert orc.ks_distance(a, b) == pytest.approx(want, abs=1e-15)
    assert orc.ks_distance(b, a) == pytest.approx(want, abs=1e-15)


def test_ks_invariant_under_monotone_maps(orc):
    rng = np.random.default_rng(5)
    a, b = rng.random(300), rng.random(200) ** 2
    d = orc.ks_distance(a, b)
    assert orc.ks_distance(np.exp(3 * a), np.exp(3 * b)) == d
    assert orc.ks_distance(-a, -b) == pytest.approx(d, abs=1e-15)
