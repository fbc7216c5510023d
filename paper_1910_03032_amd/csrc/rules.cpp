// 1D quadrature rules and Lagrange tables for the sum-factorized operators
// (Section 3.1: the Gauss point evaluation matrix B of eq. B1D and the
// differentiation matrix D of eq. D1D, here called G; nodal GLL basis of Section 3).
//
// Gauss-Legendre points: Newton on P_q with the three-term Legendre recurrence.
// GLL points: +-1 and the roots of P_p', by Newton with P_p'' taken from Legendre's
// differential equation.  Lagrange values/derivatives: barycentric weights; the
// derivative at a non-node point is phi_j(x) * sum_{m != j} 1/(x - x_m), at a node
// the classical differentiation-matrix entries.
#include <cmath>

#include "internal.h"

namespace sfem {
namespace {

// P_n(x) and P_n'(x)
void legendre(int n, double x, double &P, double &dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // (x^2 - 1) P_n' = n (x P_n - P_{n-1}), valid for |x| < 1
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

bool gauss_rule(int q, std::vector<double> &x, std::vector<double> &w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (q + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (q + 0.5));  // descending guesses
    bool ok = false;
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(q, z, P, dP);
      double dz = P / dP;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        ok = true;
        break;
      }
    }
    if (!ok) {
      // last Newton step may stall at the rounding level; accept if residual tiny
      double P, dP;
      legendre(q, z, P, dP);
      if (std::fabs(P) > 1e-13) return false;
    }
    double P, dP;
    legendre(q, z, P, dP);
    double wi = 2.0 / ((1.0 - z * z) * dP * dP);
    x[q - 1 - i] = z;
    x[i] = -z;
    w[i] = w[q - 1 - i] = wi;
  }
  if (q % 2 == 1) x[q / 2] = 0.0;
  return true;
}

bool gll_rule(int p, std::vector<double> &x, std::vector<double> &w) {
  const int n = p + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int i = 1; i <= p / 2; ++i) {
    // start from the Chebyshev-Gauss-Lobatto point, ascending from -1
    double z = -std::cos(pi * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, z, P, dP);
      double d2P = (2.0 * z * dP - p * (p + 1.0) * P) / (1.0 - z * z);
      double dz = dP / d2P;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double P, dP;
    legendre(p, z, P, dP);
    if (std::fabs(dP) > 1e-10 * (p * p + 1.0)) return false;
    x[i] = z;
    x[p - i] = -z;
  }
  if (p % 2 == 0) x[p / 2] = 0.0;
  for (int i = 0; i < n; ++i) {
    double P, dP;
    if (i == 0 || i == p) {
      P = 1.0;  // |P_p(+-1)| = 1
    } else {
      legendre(p, x[i], P, dP);
    }
    w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
  return true;
}

}  // namespace

bool make_rules(int p, int q, Rules1D &r) {
  if (p < 1 || q < 1) return false;
  r.p = p;
  r.q = q;
  if (!gll_rule(p, r.gll_x, r.gll_w)) return false;
  if (!gauss_rule(q, r.gauss_x, r.gauss_w)) return false;
  const int n = p + 1;
  // barycentric weights lambda_j = 1 / prod_{m != j} (x_j - x_m)
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int m = 0; m < n; ++m)
      if (m != j) lam[j] /= (r.gll_x[j] - r.gll_x[m]);
  r.B.assign((size_t)q * n, 0.0);
  r.G.assign((size_t)q * n, 0.0);
  for (int a = 0; a < q; ++a) {
    const double xi = r.gauss_x[a];
    int hit = -1;
    for (int m = 0; m < n; ++m)
      if (xi == r.gll_x[m]) hit = m;
    if (hit >= 0) {
      // evaluation point is a node: cardinal values, differentiation-matrix row
      double diag = 0.0;
      for (int j = 0; j < n; ++j) {
        r.B[a * n + j] = (j == hit) ? 1.0 : 0.0;
        if (j != hit) {
          double d = (lam[j] / lam[hit]) / (r.gll_x[hit] - r.gll_x[j]);
          r.G[a * n + j] = d;
          diag -= d;
        }
      }
      r.G[a * n + hit] = diag;
      continue;
    }
    double ell = 1.0;  // prod_m (xi - x_m)
    for (int m = 0; m < n; ++m) ell *= (xi - r.gll_x[m]);
    double sinv = 0.0;  // sum_m 1 / (xi - x_m)
    for (int m = 0; m < n; ++m) sinv += 1.0 / (xi - r.gll_x[m]);
    for (int j = 0; j < n; ++j) {
      double phi = ell * lam[j] / (xi - r.gll_x[j]);
      r.B[a * n + j] = phi;
      r.G[a * n + j] = phi * (sinv - 1.0 / (xi - r.gll_x[j]));
    }
  }
  return true;
}

}  // namespace sfem
