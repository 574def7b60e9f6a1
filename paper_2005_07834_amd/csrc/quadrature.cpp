// Host-side energy quadrature (Appendix D.1.b): Gauss-Legendre nodes on (0,1) by Newton
// iteration on the Legendre recurrence, and the error model used to pick the imaginary-time
// scale.
#include <cmath>
#include <vector>

#include "lrs_internal.h"

namespace lrs {

// Nodes a_j and weights w_j of the n-point Gauss-Legendre rule on (0, 1), ascending.
void gauss_legendre_01(int n, std::vector<double>& a, std::vector<double>& w) {
  a.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    // initial guess for the i-th largest root of P_n on (-1, 1)
    double x = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1.0; }
      // P_n(x) = p1, P_{n-1}(x) = p0; derivative (n/(x^2-1)) (x P_n - P_{n-1})
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = x; p0 = 1.0; }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    double wt = 2.0 / ((1.0 - x * x) * dp * dp);
    // map (-1,1) -> (0,1): root x (descending order) goes to position n-1-i
    a[n - 1 - i] = 0.5 * (x + 1.0);
    w[n - 1 - i] = 0.5 * wt;
    a[i] = 0.5 * (1.0 - x);
    w[i] = 0.5 * wt;
  }
}

// Worst relative error max_D |D * sum_j c_j exp(-D tau_j) - 1| over 512 log-spaced D of the
// time rule with scale C (tau_j = C a_j / (1 - a_j), c_j = C w_j / (1 - a_j)^2).  The samples
// are visited extremes first, and the scan stops once the error reaches `stop` (the worst
// error is a maximum, so the order does not change it).
namespace {
constexpr int kGapSamples = 512;

double rule_error(double scale, const std::vector<double>& a, const std::vector<double>& w,
                  double dmin, double dmax, double stop) {
  const int n = (int)a.size();
  std::vector<double> tau(n), c(n);
  for (int j = 0; j < n; ++j) {
    tau[j] = scale * a[j] / (1.0 - a[j]);
    c[j] = scale * w[j] / ((1.0 - a[j]) * (1.0 - a[j]));
  }
  double worst = 0;
  for (int i = 0; i < kGapSamples; ++i) {
    const int smp = i == 0 ? 0 : (i == 1 ? kGapSamples - 1 : i - 1);
    const double d = std::exp(std::log(dmin) + (std::log(dmax) - std::log(dmin)) * smp /
                                                   (kGapSamples - 1));
    double k = 0;
    for (int j = 0; j < n; ++j) k += c[j] * std::exp(-d * tau[j]);
    worst = std::fmax(worst, std::fabs(d * k - 1.0));
    if (worst >= stop) break;
  }
  return worst;
}

// The same for the even kernel Delta / (Delta^2 + omega^2) at imaginary frequency omega, with
// the coefficients times cos(omega tau_j): the worst |K (Delta^2 + omega^2) / Delta - 1|.
double rule_error_iw(double scale, const std::vector<double>& a, const std::vector<double>& w,
                     double dmin, double dmax, double omega, double stop) {
  const int n = (int)a.size();
  std::vector<double> tau(n), c(n);
  for (int j = 0; j < n; ++j) {
    tau[j] = scale * a[j] / (1.0 - a[j]);
    c[j] = scale * w[j] / ((1.0 - a[j]) * (1.0 - a[j])) * std::cos(omega * tau[j]);
  }
  double worst = 0;
  for (int i = 0; i < kGapSamples; ++i) {
    const int smp = i == 0 ? 0 : (i == 1 ? kGapSamples - 1 : i - 1);
    const double d = std::exp(std::log(dmin) + (std::log(dmax) - std::log(dmin)) * smp /
                                                   (kGapSamples - 1));
    double k = 0;
    for (int j = 0; j < n; ++j) k += c[j] * std::exp(-d * tau[j]);
    worst = std::fmax(worst, std::fabs(k * (d * d + omega * omega) / d - 1.0));
    if (worst >= stop) break;
  }
  return worst;
}
}  // namespace

namespace {
// candidate scan shared by the static and the imaginary-frequency rules (see time_auto_scale)
template <class Err>
double scan_scale(double dmin, double dmax, Err err) {
  const double g = std::sqrt(dmin * dmax);
  double best = HUGE_VAL;
  int best_j = 0;
  bool have = false;
  auto consider = [&](int j) {
    const double s = std::pow(10.0, j / 40.0) / g;
    const double stop = !have ? HUGE_VAL : (j < best_j ? std::nextafter(best, HUGE_VAL) : best);
    const double e = err(s, stop);
    if (!have || e < best || (e == best && j < best_j)) {
      best = e;
      best_j = j;
      have = true;
    }
  };
  for (int j = -80; j <= 100; j += 10) consider(j);
  for (int j = -80; j <= 100; ++j)
    if ((j + 80) % 10 != 0) consider(j);
  return std::pow(10.0, best_j / 40.0) / g;
}
}  // namespace

double time_rule_error(double scale, int n, double dmin, double dmax) {
  std::vector<double> a, w;
  gauss_legendre_01(n, a, w);
  return rule_error(scale, a, w, dmin, dmax, HUGE_VAL);
}

// Scale C = 10^(j/40) / sqrt(dmin dmax), j = -80..100, with the smallest worst error (ties to
// the smallest C).  Every tenth j is tried first, so that a good bound is known early; a
// candidate is dropped as soon as its error passes the best so far (reaches it, for a larger
// j than the best's), which leaves the choice unchanged.
double time_auto_scale(double dmin, double dmax, int n) {
  std::vector<double> a, w;
  gauss_legendre_01(n, a, w);
  return scan_scale(dmin, dmax, [&](double s, double stop) {
    return rule_error(s, a, w, dmin, dmax, stop);
  });
}

// The same scan with the imaginary-frequency error model (the static scan at omega = 0).
double time_auto_scale_iw(double dmin, double dmax, int n, double omega) {
  if (omega == 0.0) return time_auto_scale(dmin, dmax, n);
  std::vector<double> a, w;
  gauss_legendre_01(n, a, w);
  return scan_scale(dmin, dmax, [&](double s, double stop) {
    return rule_error_iw(s, a, w, dmin, dmax, omega, stop);
  });
}

}  // namespace lrs
