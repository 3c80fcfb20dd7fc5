// Host-side FP64 planner: chi-square quantiles and the parameter setting of
// PM-LSH (Lemma 3 in Section 4.3; Eq. 10 and Lemma 5 in Section 5.3), the candidate budgets
// of Algorithm 2 and Section 6.3, and the SplitMix64 generator used by the
// r_min sample of Section 5.2.
//
// The chi-square CDF is the regularised lower incomplete gamma function
// P(m/2, x/2). It is evaluated by its power series when x/2 < m/2 + 1 and
// through the complementary function Q by Legendre's continued fraction
// otherwise (Lentz's evaluation). The upper quantile solves Q(m/2, x/2) =
// alpha by Newton steps on the density, kept inside a bisection bracket.

#include <cmath>
#include <limits>

#include "internal.hpp"

namespace pmlsh {
namespace {

// P(a, x) by the series e^-x x^a sum_n x^n / Gamma(a + n + 1).
double gamma_p_series(double a, double x) {
    double term = 1.0 / a;
    double sum = term;
    for (int n = 1; n < 10000; ++n) {
        term *= x / (a + n);
        sum += term;
        if (std::fabs(term) < std::fabs(sum) * 1e-17) break;
    }
    return sum * std::exp(-x + a * std::log(x) - std::lgamma(a));
}

// Q(a, x) by the continued fraction
//   Q = e^-x x^a / Gamma(a) * 1/(x+1-a- 1(1-a)/(x+3-a- 2(2-a)/(x+5-a- ...)))
double gamma_q_cfrac(double a, double x) {
    const double tiny = 1e-300;
    double b = x + 1.0 - a;
    double c = 1.0 / tiny;
    double d = 1.0 / b;
    double h = d;
    for (int i = 1; i < 10000; ++i) {
        double an = -i * (i - a);
        b += 2.0;
        d = an * d + b;
        if (std::fabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (std::fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double delta = d * c;
        h *= delta;
        if (std::fabs(delta - 1.0) < 1e-17) break;
    }
    return std::exp(-x + a * std::log(x) - std::lgamma(a)) * h;
}

double chi2_sf(double x, int m) {
    if (x <= 0.0) return 1.0;
    if (std::isinf(x)) return 0.0;
    double a = 0.5 * m, y = 0.5 * x;
    if (y < a + 1.0) return 1.0 - gamma_p_series(a, y);
    return gamma_q_cfrac(a, y);
}

double chi2_pdf(double x, int m) {
    if (x <= 0.0) return 0.0;
    double a = 0.5 * m;
    return std::exp((a - 1.0) * std::log(x) - 0.5 * x - a * std::log(2.0) - std::lgamma(a));
}

}  // namespace

double chi2_cdf(double x, int m) {
    if (x <= 0.0) return 0.0;
    if (std::isinf(x)) return 1.0;
    double a = 0.5 * m, y = 0.5 * x;
    if (y < a + 1.0) return gamma_p_series(a, y);
    return 1.0 - gamma_q_cfrac(a, y);
}

double chi2_upper_quantile(double alpha, int m) {
    // bracket [lo, hi] with sf(lo) > alpha >= sf(hi)
    double lo = 0.0, hi = std::max(1.0, (double)m);
    while (chi2_sf(hi, m) > alpha) { lo = hi; hi *= 2.0; }
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double f = chi2_sf(x, m) - alpha;
        if (f > 0) lo = x; else hi = x;
        double p = chi2_pdf(x, m);
        double nx = (p > 0) ? x + f / p : 0.5 * (lo + hi);  // d(sf)/dx = -pdf
        if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
        if (std::fabs(nx - x) <= 1e-15 * x || hi - lo <= 1e-15 * hi) { x = nx; break; }
        x = nx;
    }
    return x;
}

uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void plan_params(int64_t n, int m, int k, double c, double confidence,
                 double beta, pmlsh_plan* out) {
    if (n < 1) fail(PMLSH_EINVAL, "n must be >= 1");
    if (m < 1 || m > PMLSH_MAX_M) fail(PMLSH_EINVAL, "m must be in 1..16");
    if (k < 1) fail(PMLSH_EINVAL, "k must be >= 1");
    if (!std::isfinite(c) || !(c > 1.0)) fail(PMLSH_EINVAL, "c must be finite and > 1");
    if (!(confidence > 0.0 && confidence < 1.0))
        fail(PMLSH_EINVAL, "confidence must lie in (0, 1)");
    if (std::isnan(beta) || beta > 1.0) fail(PMLSH_EINVAL, "beta must be <= 1 (or < 0 for the default)");
    const double alpha1 = 1.0 - confidence;
    const double t2 = chi2_upper_quantile(alpha1, m);          // Eq. 10, first line
    const double alpha2 = chi2_cdf(t2 / (c * c), m);           // Eq. 10, second line
    const double b = beta < 0.0 ? 2.0 * alpha2 : beta;         // Lemma 5
    out->t = std::sqrt(t2);
    out->alpha1 = alpha1;
    out->alpha2 = alpha2;
    out->beta = b;
    int64_t B = (int64_t)std::ceil(b * (double)n) + k;
    out->budget = B < n ? B : n;
    out->acp_budget = (int64_t)std::ceil(b * ((double)n * (double)(n - 1) / 2.0)) + k;
}

}  // namespace pmlsh
