"""Chi-square distribution and the PM-LSH parameter setting (oracle, FP64).

Lemma 1 (Section 3.2): for two points at distance r, r'^2 / r^2 follows
chi^2(m) when the m projection vectors have i.i.d. N(0,1) entries.
Lemma 3 (Section 4.3) uses the *upper* quantile chi^2_alpha(m), defined by
  integral_{chi^2_alpha(m)}^{inf} f(x; m) dx = alpha.
Eq. 10 (Section 5.3) ties the radius factor t to two probabilities:
  t^2 = chi^2_{alpha1}(m)  and  t^2 = c^2 * chi^2_{1-alpha2}(m).

The CDF is written from its closed form (regularised lower incomplete gamma
function at half-integer / integer order):
  m even:  P(x; m) = 1 - exp(-y) * sum_{j=0}^{m/2-1} y^j / j!
  m odd :  P(x; m) = erf(sqrt y) - exp(-y) * sum_{j=1}^{(m-1)/2} y^{j-1/2} / Gamma(j+1/2)
with y = x/2; the survival function 1-P is summed directly in the same
terms so that small upper tails keep their relative accuracy.
"""

from __future__ import annotations

import math


def _series(y: float, m: int) -> float:
    """exp(-y) times the finite sum that appears in both closed forms."""
    if y == 0.0:
        return 1.0 if m % 2 == 0 else 0.0
    ly = math.log(y)
    total = 0.0
    if m % 2 == 0:
        for j in range(m // 2):
            total += math.exp(j * ly - y - math.lgamma(j + 1.0))
    else:
        for j in range(1, (m - 1) // 2 + 1):
            total += math.exp((j - 0.5) * ly - y - math.lgamma(j + 0.5))
    return total


def cdf(x: float, m: int) -> float:
    """P[X <= x] for X ~ chi^2(m)."""
    if m < 1:
        raise ValueError("m must be >= 1")
    if x <= 0.0:
        return 0.0
    if math.isinf(x):
        return 1.0
    y = 0.5 * x
    if m % 2 == 0:
        return 1.0 - _series(y, m)
    return math.erf(math.sqrt(y)) - _series(y, m)


def sf(x: float, m: int) -> float:
    """P[X > x] for X ~ chi^2(m)."""
    if m < 1:
        raise ValueError("m must be >= 1")
    if x <= 0.0:
        return 1.0
    if math.isinf(x):
        return 0.0
    y = 0.5 * x
    if m % 2 == 0:
        return _series(y, m)
    return math.erfc(math.sqrt(y)) + _series(y, m)


def upper_quantile(alpha: float, m: int) -> float:
    """chi^2_alpha(m): the x with P[X > x] = alpha (Lemma 3), by bisection.

    sf is strictly decreasing on (0, inf); the bracket is grown until it
    holds the root, then halved until the interval is below 1e-13 relative.
    """
    if not (0.0 < alpha < 1.0):
        raise ValueError("alpha must lie in (0, 1)")
    lo, hi = 0.0, max(1.0, float(m))
    while sf(hi, m) > alpha:
        lo, hi = hi, 2.0 * hi
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if sf(mid, m) > alpha:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-13 * hi:
            break
    return 0.5 * (lo + hi)


def radius_factor(alpha1: float, m: int) -> float:
    """t = sqrt(chi^2_{alpha1}(m)), first line of Eq. 10."""
    return math.sqrt(upper_quantile(alpha1, m))


def alpha2(alpha1: float, c: float, m: int) -> float:
    """alpha2 solving the second line of Eq. 10.

    t^2 / c^2 = chi^2_{1-alpha2}(m) means P[X > t^2/c^2] = 1 - alpha2,
    i.e. alpha2 = P[X <= t^2 / c^2].
    """
    t2 = upper_quantile(alpha1, m)
    return cdf(t2 / (c * c), m)


def default_beta(alpha1: float, c: float, m: int) -> float:
    """beta = 2 * alpha2, the setting of Lemma 5 (Section 5.3)."""
    return 2.0 * alpha2(alpha1, c, m)


def ann_budget(beta: float, n: int, k: int) -> int:
    """B = beta*n + k candidates (Alg. 2); beta*n rounded up, capped at n."""
    return min(n, int(math.ceil(beta * n)) + k)


def acp_budget(beta: float, n: int, k: int) -> int:
    """T = beta * n(n-1)/2 + k candidate pairs (Section 6.3), rounded up."""
    return int(math.ceil(beta * (n * (n - 1) / 2.0))) + k
