// Gauss-Lobatto-Legendre nodes, weights and derivative matrix of degree P,
// evaluated at compile time with the construction of the host tables: the
// interior nodes are the roots of P_P', bracketed on a grid and refined by
// bisection; the weights are 2 / (P (P+1) P_P(x)^2); the derivative matrix
// is the barycentric one with rows summing to zero (Sec. 6, degree P).
//
// Kernels that contract with the derivative matrix use these values as
// compile-time constants: a constant is rebuilt in place wherever it is
// used, so the matrix holds no registers between uses.
#pragma once

namespace sisdc {

namespace gllc {

constexpr double absd(double v) { return v < 0.0 ? -v : v; }

// P_n(x) and P_n'(x) (three-term recurrence; the derivative from
// (1 - x^2) P_n' = n (P_{n-1} - x P_n) inside (-1, 1))
constexpr void legendre_pd(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  if (absd(x) < 1.0)
    dp = n * (p0 - x * p1) / (1.0 - x * x);
  else
    dp = (x > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0)) * 0.5 * n * (n + 1.0);
}

constexpr double dleg(int n, double x) {
  double p = 0.0, dp = 0.0;
  legendre_pd(n, x, p, dp);
  return dp;
}

}  // namespace gllc

template <int P>
struct GLLConst {
  static constexpr int N1 = P + 1;
  double x[N1] = {};
  double w[N1] = {};
  double D[N1][N1] = {};
  constexpr GLLConst() {
    constexpr int grid = 4000;
    x[0] = -1.0;
    int nr = 1;
    double xl = -1.0, fl = gllc::dleg(P, -1.0);
    for (int k = 1; k <= grid && nr < P; ++k) {
      const double xr = -1.0 + 2.0 * k / grid;
      const double fr = gllc::dleg(P, xr);
      if (fl == 0.0 && xl > -1.0) {
        x[nr++] = xl;
      } else if ((fl < 0.0 && fr > 0.0) || (fl > 0.0 && fr < 0.0)) {
        double lo = xl, hi = xr, flo = fl;
        for (int it = 0; it < 200; ++it) {
          const double mid = 0.5 * (lo + hi);
          if (mid <= lo || mid >= hi) break;
          const double fm = gllc::dleg(P, mid);
          if ((fm < 0.0) == (flo < 0.0)) {
            lo = mid;
            flo = fm;
          } else {
            hi = mid;
          }
        }
        x[nr++] = 0.5 * (lo + hi);
      }
      xl = xr;
      fl = fr;
    }
    x[P] = 1.0;
    for (int j = 0; j < N1; ++j) {
      double p = 0.0, dp = 0.0;
      gllc::legendre_pd(P, x[j], p, dp);
      w[j] = 2.0 / (P * (P + 1.0) * p * p);
    }
    double lam[N1] = {};
    for (int j = 0; j < N1; ++j) {
      lam[j] = 1.0;
      for (int k = 0; k < N1; ++k)
        if (k != j) lam[j] /= (x[j] - x[k]);
    }
    for (int i = 0; i < N1; ++i) {
      double s = 0.0;
      for (int j = 0; j < N1; ++j)
        if (j != i) {
          D[i][j] = (lam[j] / lam[i]) / (x[i] - x[j]);
          s += D[i][j];
        }
      D[i][i] = -s;
    }
  }
};

template <int P>
inline constexpr GLLConst<P> kGLL{};

}  // namespace sisdc
