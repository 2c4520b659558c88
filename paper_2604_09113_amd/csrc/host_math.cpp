// Small host-side polynomial tables: Legendre-based quadrature points and the
// Lagrange/Bernstein values the kernels read.  Standard textbook methods:
// Newton iteration on the Legendre three-term recurrence for Gauss and
// Gauss-Lobatto points, product formulas for Lagrange polynomials.
#include <cmath>
#include <vector>

#include "internal.h"

namespace lbddc {

// P_n(x) and P_n'(x) on [-1, 1] from the three-term recurrence.
static void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

std::vector<double> gll_points(int p) {
  std::vector<double> x(p + 1);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double xi = -std::cos(M_PI * i / p);  // Chebyshev-Lobatto start
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, xi, P, dP);
      // P'' from the Legendre equation (1 - x^2) P'' = 2x P' - p(p+1) P
      double d2P = (2.0 * xi * dP - p * (p + 1.0) * P) / (1.0 - xi * xi);
      double dx = dP / d2P;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    x[i] = xi;
  }
  for (auto& v : x) v = 0.5 * (v + 1.0);
  return x;
}

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double xi = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double P = 0, dP = 1;
    for (int it = 0; it < 100; ++it) {
      legendre(n, xi, P, dP);
      double dx = P / dP;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    legendre(n, xi, P, dP);
    x[n - 1 - i] = 0.5 * (xi + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - xi * xi) * dP * dP);  // 2/((1-x^2)P'^2) halved for [0,1]
  }
}

double lagrange_value(const std::vector<double>& nodes, int a, double x) {
  double v = 1.0;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != a) v *= (x - nodes[m]) / (nodes[a] - nodes[m]);
  return v;
}

double lagrange_derivative(const std::vector<double>& nodes, int a, double x) {
  double s = 0.0;
  for (size_t l = 0; l < nodes.size(); ++l) {
    if ((int)l == a) continue;
    double term = 1.0 / (nodes[a] - nodes[l]);
    for (size_t m = 0; m < nodes.size(); ++m)
      if ((int)m != a && m != l) term *= (x - nodes[m]) / (nodes[a] - nodes[m]);
    s += term;
  }
  return s;
}

static double binom(int n, int k) {
  double b = 1.0;
  for (int i = 1; i <= k; ++i) b = b * (n - k + i) / i;
  return b;
}

double bernstein_value(int m, int a, double x) {
  if (a < 0 || a > m) return 0.0;
  return binom(m, a) * std::pow(x, a) * std::pow(1.0 - x, m - a);
}

double bernstein_derivative(int m, int a, double x) {
  if (m == 0) return 0.0;
  return m * (bernstein_value(m - 1, a - 1, x) - bernstein_value(m - 1, a, x));
}

}  // namespace lbddc
