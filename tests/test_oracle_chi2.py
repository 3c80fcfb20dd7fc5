"""Pins of the oracle's chi-square math (Lemma 1, Lemma 3, Eq. 10, Lemma 5).

The oracle's closed forms are checked against SciPy's independent
implementation of the chi-square distribution, against special cases that
have textbook closed forms, and against the one parameter value the paper
prints that Eq. 10 reproduces.
"""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import chi2


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 8, 15, 16, 31])
def test_cdf_sf_match_scipy(m):
    xs = np.concatenate([np.linspace(0.01, 4 * m + 40, 97), [1e-6, 0.5 * m, m]])
    for x in xs:
        assert chi2.cdf(x, m) == pytest.approx(stats.chi2.cdf(x, m), abs=1e-14)
        ref_sf = stats.chi2.sf(x, m)
        assert chi2.sf(x, m) == pytest.approx(ref_sf, rel=1e-11, abs=1e-300)


@pytest.mark.parametrize("m", [1, 2, 3, 15, 16])
@pytest.mark.parametrize("alpha", [0.01, 0.05, 0.1, 1 / math.e, 0.5, 0.9, 0.95])
def test_upper_quantile_matches_scipy(m, alpha):
    assert chi2.upper_quantile(alpha, m) == pytest.approx(
        stats.chi2.isf(alpha, m), rel=1e-11)


def test_m1_is_erf_of_half_x():
    # chi^2(1) is the square of a standard normal: P[Z^2 <= x] = erf(sqrt(x/2))
    for x in [0.1, 1.0, 2.7, 9.0]:
        assert chi2.cdf(x, 1) == pytest.approx(math.erf(math.sqrt(x / 2)),
                                               abs=1e-15)


def test_m2_closed_form_quantile():
    # chi^2(2) is exponential with mean 2: upper quantile = -2 ln(alpha).
    for a in [0.05, 0.1, 1 / math.e, 0.7]:
        assert chi2.upper_quantile(a, 2) == pytest.approx(-2 * math.log(a),
                                                          rel=1e-12)
    # so alpha1 = 1/e gives t^2 = 2, and Eq. 10 gives alpha2 = 1 - exp(-1/c^2)
    assert chi2.radius_factor(1 / math.e, 2) ** 2 == pytest.approx(2.0, rel=1e-12)
    for c in [1.2, 1.5, 2.0]:
        assert chi2.alpha2(1 / math.e, c, 2) == pytest.approx(
            1 - math.exp(-1 / c ** 2), rel=1e-12)


def test_eq10_reproduces_printed_cp_alpha2():
    # Section 7.1 (CP parameter settings) prints alpha2 = 0.0024 for m = 15,
    # alpha1 = 1/e. Eq. 10 gives 0.002444 with c = 2 (the square root of the
    # CP default ratio c = 4, Theorem 1's c^2 guarantee), which rounds to the
    # printed value.
    a2 = chi2.alpha2(1 / math.e, 2.0, 15)
    assert round(a2, 4) == 0.0024
    assert a2 == pytest.approx(0.002444, abs=5e-7)


def test_eq10_round_trip():
    # t^2 = c^2 chi^2_{1-alpha2}(m) must hold for the alpha2 returned.
    for m in [2, 7, 15]:
        for c in [1.2, 1.5, 2.0, 3.0]:
            t2 = chi2.upper_quantile(1 / math.e, m)
            a2 = chi2.alpha2(1 / math.e, c, m)
            assert c * c * stats.chi2.isf(1 - a2, m) == pytest.approx(t2, rel=1e-9)


def test_lemma5_default_beta_and_budgets():
    b = chi2.default_beta(1 / math.e, 1.5, 15)
    assert b == pytest.approx(2 * stats.chi2.cdf(stats.chi2.isf(1 / math.e, 15)
                                                 / 2.25, 15), rel=1e-10)
    assert chi2.ann_budget(0.1, 10_000, 10) == 1010
    assert chi2.ann_budget(1.0, 100, 10) == 100          # capped at n
    assert chi2.ann_budget(0.0, 100, 7) == 7
    assert chi2.acp_budget(0.0, 100, 5) == 5
    assert chi2.acp_budget(0.01, 101, 3) == math.ceil(0.01 * 101 * 50) + 3


def test_confidence_point_of_parity_workload():
    # confidence 0.9 read as Pr[E1] = 1 - alpha1: alpha1 = 0.1 -> t^2 is the
    # upper 10 % point of chi^2(15)
    assert chi2.radius_factor(0.1, 15) ** 2 == pytest.approx(
        stats.chi2.ppf(0.9, 15), rel=1e-11)


def test_invalid_arguments():
    with pytest.raises(ValueError):
        chi2.upper_quantile(0.0, 15)
    with pytest.raises(ValueError):
        chi2.upper_quantile(1.0, 15)
    with pytest.raises(ValueError):
        chi2.cdf(1.0, 0)


def test_budgets_round_beta_n_up():
    assert chi2.ann_budget(0.0015, 1001, 1) == 3      # ceil(1.5015) + 1
    assert chi2.acp_budget(0.001, 100, 2) == 7        # ceil(4.95) + 2
