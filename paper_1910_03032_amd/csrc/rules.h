// Compile-time 1D quadrature rules and Lagrange tables (Section 3.1: the Gauss-point
// evaluation matrix B of eq. B1D and the differentiation matrix of eq. D1D, here G;
// nodal GLL basis of Section 3).
//
// Everything is constexpr, so the kernels see B and G as literal constants of their
// compile-time order p (the loop bounds and the tables are both known at compile
// time), and the host copies the very same compile-time values.
//
//  * Gauss-Legendre points: Newton on P_q (three-term recurrence for P_q, P_q'),
//    starting from cos(pi (i + 3/4) / (q + 1/2)); weights 2 / ((1 - x^2) P_q'(x)^2).
//  * GLL points: +-1 and the roots of P_p', Newton with P_p'' taken from Legendre's
//    differential equation, starting from the Chebyshev-Gauss-Lobatto points;
//    weights 2 / (p (p + 1) P_p(x)^2).
//  * Lagrange basis on the GLL points with barycentric weights; at a point that is
//    not a node phi_j'(x) = phi_j(x) sum_{m != j} 1 / (x - x_m); at a node, the
//    classical differentiation-matrix entries.
#pragma once

namespace sfem {
namespace rules {

constexpr double kPi = 3.14159265358979323846;

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// cos(x) for x in [0, pi] by its Taylor series (only used for Newton start values)
constexpr double ccos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

struct PdP {
  double P, dP, Pm1;
};

// P_n(x), P_n'(x) (for |x| < 1) and P_{n-1}(x)
constexpr PdP legendre(int n, double x) {
  double p0 = 1.0, p1 = x;
  if (n == 0) return PdP{1.0, 0.0, 0.0};
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return PdP{p1, n * (x * p1 - p0) / (x * x - 1.0), p0};
}

template <int Q>
struct GaussRule {
  double x[Q];
  double w[Q];
};

template <int Q>
constexpr GaussRule<Q> gauss() {
  GaussRule<Q> r{};
  for (int i = 0; i < (Q + 1) / 2; ++i) {
    double z = ccos(kPi * (i + 0.75) / (Q + 0.5));
    for (int it = 0; it < 100; ++it) {
      const PdP v = legendre(Q, z);
      const double dz = v.P / v.dP;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    const PdP v = legendre(Q, z);
    const double w = 2.0 / ((1.0 - z * z) * v.dP * v.dP);
    r.x[Q - 1 - i] = z;
    r.x[i] = -z;
    r.w[i] = w;
    r.w[Q - 1 - i] = w;
  }
  if (Q % 2 == 1) r.x[Q / 2] = 0.0;
  return r;
}

template <int P>
struct GllRule {
  double x[P + 1];
  double w[P + 1];
};

template <int P>
constexpr GllRule<P> gll() {
  GllRule<P> r{};
  r.x[0] = -1.0;
  r.x[P] = 1.0;
  for (int i = 1; i <= P / 2; ++i) {
    double z = -ccos(kPi * i / P);
    for (int it = 0; it < 100; ++it) {
      const PdP v = legendre(P, z);
      const double d2P = (2.0 * z * v.dP - P * (P + 1.0) * v.P) / (1.0 - z * z);
      const double dz = v.dP / d2P;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    r.x[i] = z;
    r.x[P - i] = -z;
  }
  if (P % 2 == 0) r.x[P / 2] = 0.0;
  for (int i = 0; i <= P; ++i) {
    const double Pv = (i == 0 || i == P) ? 1.0 : legendre(P, r.x[i]).P;
    r.w[i] = 2.0 / (P * (P + 1.0) * Pv * Pv);
  }
  return r;
}

// B[a][i] = phi_i(xi_a), G[a][i] = phi_i'(xi_a) for the p+1 GLL nodes and q Gauss points
template <int P, int Q>
struct Tables {
  double B[Q][P + 1];
  double G[Q][P + 1];
};

template <int P, int Q>
constexpr Tables<P, Q> tables() {
  constexpr int N = P + 1;
  const GllRule<P> nodes = gll<P>();
  const GaussRule<Q> pts = gauss<Q>();
  double lam[N] = {};
  for (int j = 0; j < N; ++j) {
    lam[j] = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != j) lam[j] /= (nodes.x[j] - nodes.x[m]);
  }
  Tables<P, Q> t{};
  for (int a = 0; a < Q; ++a) {
    const double xi = pts.x[a];
    int hit = -1;
    for (int m = 0; m < N; ++m)
      if (xi == nodes.x[m]) hit = m;
    if (hit >= 0) {
      double diag = 0.0;
      for (int j = 0; j < N; ++j) {
        t.B[a][j] = (j == hit) ? 1.0 : 0.0;
        if (j != hit) {
          const double d = (lam[j] / lam[hit]) / (nodes.x[hit] - nodes.x[j]);
          t.G[a][j] = d;
          diag -= d;
        }
      }
      t.G[a][hit] = diag;
      continue;
    }
    double ell = 1.0, sinv = 0.0;
    for (int m = 0; m < N; ++m) {
      ell *= (xi - nodes.x[m]);
      sinv += 1.0 / (xi - nodes.x[m]);
    }
    for (int j = 0; j < N; ++j) {
      const double phi = ell * lam[j] / (xi - nodes.x[j]);
      t.B[a][j] = phi;
      t.G[a][j] = phi * (sinv - 1.0 / (xi - nodes.x[j]));
    }
  }
  return t;
}

// Compile-time instances (one per order, q = p + 2).
template <int P>
struct Const {
  static constexpr Tables<P, P + 2> tab = tables<P, P + 2>();
  static constexpr GaussRule<P + 2> gauss_rule = gauss<P + 2>();
  static constexpr GllRule<P> gll_rule = gll<P>();
};

}  // namespace rules
}  // namespace sfem
