// Confidence bands of the on-line statistics (paper Sec. 5.2 schema iii and
// the experiments of Sec. 5: mean, variance and a confidence interval per
// sample time over the instances).  Host-side: the half-width of the
// two-sided Student-t interval at a given level,
//   w = t_{(1+level)/2, n-1} * sqrt(var / n),
// from the per-sample n and the unbiased variance the runs produce.
//
// The t quantile is the inverse of the Student-t distribution function,
// written through the regularized incomplete beta function:
//   for t >= 0, P(T > t) = I_x(nu/2, 1/2) / 2 with x = nu / (nu + t^2).
// I_x(a, b) is evaluated with its continued fraction (modified Lentz
// algorithm, extended precision), and the quantile is found by Newton
// steps on t safeguarded by bisection; it is accurate to about 1e-12.
#include <cmath>
#include <cstdint>
#include <limits>

#include "../../include/cwcssa.h"
#include "runtime.h"

namespace {

// continued fraction of I_x(a, b) (valid for x < (a + 1) / (a + b + 2)),
// given x and y = 1 - x (both exact to the last bit).  Its first term
// 1 - (a + b) x / (a + 1) is written, for x >= 1/2, as
// ((1 - b) + (a + b) y) / (a + 1), free of cancellation when x is close to
// 1 and a is large; the recurrence runs in extended precision.
double beta_cf(double a_, double b_, double x_, double y_)
{
    typedef long double L;
    const L a = a_, b = b_, x = x_, y = y_;
    const L tiny = 1e-300L, eps = 1e-19L;
    L c = 1.0L;
    L d = x < 0.5L ? 1.0L - (a + b) * x / (a + 1.0L) : ((1.0L - b) + (a + b) * y) / (a + 1.0L);
    if (std::fabs(d) < tiny) d = tiny;
    d = 1.0L / d;
    L h = d;
    for (int m = 1; m <= 20000; ++m) {
        const L m2 = 2.0L * m;
        L aa = m * (b - m) * x / ((a + m2 - 1.0L) * (a + m2));
        d = 1.0L + aa * d;
        if (std::fabs(d) < tiny) d = tiny;
        c = 1.0L + aa / c;
        if (std::fabs(c) < tiny) c = tiny;
        d = 1.0L / d;
        h *= d * c;
        aa = -(a + m) * (a + b + m) * x / ((a + m2) * (a + m2 + 1.0L));
        d = 1.0L + aa * d;
        if (std::fabs(d) < tiny) d = tiny;
        c = 1.0L + aa / c;
        if (std::fabs(c) < tiny) c = tiny;
        d = 1.0L / d;
        const L del = d * c;
        h *= del;
        if (std::fabs(del - 1.0L) < eps) break;
    }
    return (double)h;
}

// ln Gamma(a + 1/2) - ln Gamma(a).  For large a the difference of two
// lgamma values loses about log10(a ln a) digits, so there it is written
// from Stirling's series (truncation below 2e-15 for a >= 20), ln Gamma(z) = (z - 1/2) ln z - z + ln(2 pi)/2 +
// 1/(12 z) - 1/(360 z^3) + 1/(1260 z^5) - 1/(1680 z^7) + ..., with the
// leading terms combined exactly:
//   (1/2) ln a + a log1p(1/(2a)) - 1/2 + S(a + 1/2) - S(a).
double lgamma_half_step(double a)
{
    if (a < 20.0) return std::lgamma(a + 0.5) - std::lgamma(a);
    auto S = [](double z) {
        const double z2 = z * z;
        return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0 - 1.0 / (1680.0 * z2)) / z2) / z2) / z;
    };
    return 0.5 * std::log(a) + (a * std::log1p(0.5 / a) - 0.5) + (S(a + 0.5) - S(a));
}

// upper tail P(T > t) of Student's t with nu degrees of freedom, t >= 0:
// I_x(nu/2, 1/2) / 2 with x = nu / (nu + t^2)
double t_upper(double t, double nu)
{
    if (t <= 0.0) return 0.5;
    const double a = 0.5 * nu, b = 0.5;
    const double r = t * t / nu;
    const double lnx = -std::log1p(r);                 // ln x
    const double ln1mx = std::log(r) + lnx;            // ln(1 - x) = ln(r / (1 + r))
    const double x = std::exp(lnx), y = -std::expm1(lnx);
    // ln(1 / B(a, b)) = ln Gamma(a + 1/2) - ln Gamma(a) - ln Gamma(1/2)
    const double lfront = lgamma_half_step(a) - 0.5 * std::log(M_PI) + a * lnx + b * ln1mx;
    const double front = std::exp(lfront);
    double I;
    if (x < (a + 1.0) / (a + b + 2.0)) I = front * beta_cf(a, b, x, y) / a;
    else I = 1.0 - front * beta_cf(b, a, y, x) / b;
    return 0.5 * I;
}

// density of Student's t
double t_pdf(double t, double nu)
{
    const double lc = lgamma_half_step(0.5 * nu) - 0.5 * std::log(nu * M_PI);
    return std::exp(lc - 0.5 * (nu + 1.0) * std::log1p(t * t / nu));
}

}  // namespace

namespace cwc {

// t with P(T > t) = q (0 < q < 0.5), nu > 0
double student_t_upper_quantile(double q, double nu)
{
    double lo = 0.0, hi = 1.0;
    while (t_upper(hi, nu) > q) {
        lo = hi;
        hi *= 2.0;
        if (hi > 1e300) return std::numeric_limits<double>::infinity();
    }
    double t = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double f = t_upper(t, nu) - q;       // decreasing in t
        if (f > 0) lo = t; else hi = t;
        const double step = f / t_pdf(t, nu);      // Newton on -F
        double tn = t + step;
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (std::fabs(tn - t) <= 1e-15 * std::fabs(tn) || hi - lo <= 1e-15 * hi) return tn;
        t = tn;
    }
    return t;
}

}  // namespace cwc

extern "C" cwc_status cwc_stats_confidence(const double *var, const int64_t *n, int64_t rows,
                                           int32_t n_cells, double level, double *half_width)
{
    if ((rows > 0 && (!var || !n || !half_width)) || rows < 0 || n_cells < 1)
        return cwc::set_err(CWC_E_INVALID, "bad arguments");
    if (!(level > 0.0 && level < 1.0)) return cwc::set_err(CWC_E_INVALID, "level must be in (0, 1)");
    const double q = 0.5 * (1.0 - level);
    const double nan = std::numeric_limits<double>::quiet_NaN();
    int64_t last_n = -1;
    double tq = nan;
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t nr = n[r];
        if (nr != last_n) {
            tq = nr >= 2 ? cwc::student_t_upper_quantile(q, (double)(nr - 1)) : nan;
            last_n = nr;
        }
        for (int32_t c = 0; c < n_cells; ++c) {
            const double v = var[r * (int64_t)n_cells + c];
            half_width[r * (int64_t)n_cells + c] =
                nr >= 2 ? tq * std::sqrt(v / (double)nr) : nan;
        }
    }
    return CWC_OK;
}
