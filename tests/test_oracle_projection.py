"""Pins of the oracle's projection against Lemmas 1-3 (Section 3.2, 4.3).

For a fixed pair at distance r and many independent hash matrices A with
N(0,1) entries, r'^2 / r^2 must follow chi^2(m) (Lemma 1), r'^2/m must be an
unbiased estimate of r^2 (Lemma 2) and Pr[r' > t r] must equal alpha when
t^2 is the upper alpha quantile (Lemma 3). A transposed, truncated or
mis-scaled projection fails these distributional checks.
"""

import math

import numpy as np
from scipy import stats

from oracle import ann, chi2

M = 15
D = 64
TRIALS = 4000


def _ratios(seed=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    o1 = rng.standard_normal(D).astype(np.float32)
    o2 = (o1 + 0.3 * rng.standard_normal(D)).astype(np.float32)
    r2 = float(np.sum((o1.astype(np.float64) - o2) ** 2))
    out = np.empty(TRIALS)
    for s in range(TRIALS):
        A = rng.standard_normal((M, D)).astype(np.float32)
        p = ann.project(np.stack([o1, o2]), A)
        out[s] = float(np.sum((p[0] - p[1]) ** 2)) / r2
    return out


def test_lemma1_projected_ratio_is_chi2():
    x = _ratios()
    ks = stats.kstest(x, stats.chi2(M).cdf)
    assert ks.pvalue > 1e-3
    # wrong degrees of freedom must be rejected by the same test
    assert stats.kstest(x, stats.chi2(M - 2).cdf).pvalue < 1e-6


def test_lemma2_estimator_unbiased():
    x = _ratios(seed=11)
    # mean of chi^2(m)/m is 1 with standard error sqrt(2/m)/sqrt(TRIALS)
    se = math.sqrt(2.0 / M) / math.sqrt(TRIALS)
    assert abs(np.mean(x) / M - 1.0) < 4 * se


def test_lemma3_tail_probabilities():
    x = _ratios(seed=13)
    for alpha in [0.1, 1 / math.e]:
        t2 = chi2.upper_quantile(alpha, M)
        p_hi = np.mean(x > t2)                       # P2: r' > r sqrt(chi2_a)
        lo2 = chi2.upper_quantile(1 - alpha, M)
        p_lo = np.mean(x < lo2)                      # P1: r' < r sqrt(chi2_{1-a})
        se = math.sqrt(alpha * (1 - alpha) / TRIALS)
        assert abs(p_hi - alpha) < 4 * se
        assert abs(p_lo - alpha) < 4 * se


def test_projection_shape_and_linearity():
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.standard_normal((5, 9)).astype(np.float32)
    A = rng.standard_normal((4, 9)).astype(np.float32)
    P = ann.project(X, A)
    assert P.shape == (5, 4)
    # row i, column j is the dot product of point i with hash vector j
    assert P[2, 3] == sum(float(A[3, c]) * float(X[2, c]) for c in range(9)) \
        or abs(P[2, 3] - sum(float(A[3, c]) * float(X[2, c])
                             for c in range(9))) < 1e-12
