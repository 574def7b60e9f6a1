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

// Worst relative error max_D |D * sum_j c_j exp(-D tau_j) - 1| over 512 log-spaced D.
double time_rule_error(double scale, int n, double dmin, double dmax) {
  std::vector<double> a, w;
  gauss_legendre_01(n, a, w);
  double worst = 0;
  const int ns = 512;
  for (int s = 0; s < ns; ++s) {
    double d = std::exp(std::log(dmin) + (std::log(dmax) - std::log(dmin)) * s / (ns - 1));
    double k = 0;
    for (int j = 0; j < n; ++j) {
      double tau = scale * a[j] / (1.0 - a[j]);
      double c = scale * w[j] / ((1.0 - a[j]) * (1.0 - a[j]));
      k += c * std::exp(-d * tau);
    }
    worst = std::fmax(worst, std::fabs(d * k - 1.0));
  }
  return worst;
}

double time_auto_scale(double dmin, double dmax, int n) {
  double g = std::sqrt(dmin * dmax);
  double best = -1, best_s = 1.0 / g;
  for (int j = -80; j <= 100; ++j) {
    double s = std::pow(10.0, j / 40.0) / g;
    double e = time_rule_error(s, n, dmin, dmax);
    if (best < 0 || e < best) {
      best = e;
      best_s = s;
    }
  }
  return best_s;
}

}  // namespace lrs
