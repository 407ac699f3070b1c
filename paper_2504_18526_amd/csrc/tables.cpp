// Reference-element and collocation tables, computed on the host once per
// level.  Roots are bracketed on a fine grid and refined by bisection, which
// needs nothing but polynomial evaluation:
//   GLL nodes      : -1, +1 and the roots of P_P'            (Sec. 6, degree P)
//   Radau right    : the roots of P_M - P_{M-1} on (-1, 1], mapped to [0, 1]
//                    (Sec. 3, Radau Right nodes)
//   Gauss-Legendre : roots of P_n, weights 2 / ((1 - x^2) P_n'(x)^2)
//   w^nn           : eq. (nn_weights), integrated with Gauss-Legendre
#include "tables.hpp"

#include <cmath>
#include <functional>

namespace sisdc {

// P_n(x) and P_n'(x) by the three-term recurrence.
static void legendre_pd(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n), valid inside (-1, 1)
  if (std::fabs(x) < 1.0) dp = n * (p0 - x * p1) / (1.0 - x * x);
  else dp = (x > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0)) * 0.5 * n * (n + 1.0);
}

// All roots of f strictly inside (a, b), by sign changes on a grid + bisection.
static std::vector<double> roots(const std::function<double(double)>& f, double a, double b, int grid) {
  std::vector<double> r;
  double xl = a, fl = f(a);
  for (int k = 1; k <= grid; ++k) {
    double xr = a + (b - a) * k / grid;
    double fr = f(xr);
    if (fl == 0.0 && xl > a) r.push_back(xl);
    else if ((fl < 0.0 && fr > 0.0) || (fl > 0.0 && fr < 0.0)) {
      double lo = xl, hi = xr, flo = fl;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm = f(mid);
        if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else hi = mid;
      }
      r.push_back(0.5 * (lo + hi));
    }
    xl = xr;
    fl = fr;
  }
  return r;
}

void gll(int P, std::vector<double>& x, std::vector<double>& w) {
  x.assign(1, -1.0);
  auto dP = [P](double t) { double p, dp; legendre_pd(P, t, p, dp); return dp; };
  std::vector<double> in = roots(dP, -1.0, 1.0, 4000);
  for (double t : in) x.push_back(t);
  x.push_back(1.0);
  w.resize(x.size());
  for (size_t j = 0; j < x.size(); ++j) {
    double p, dp;
    legendre_pd(P, x[j], p, dp);
    w[j] = 2.0 / (P * (P + 1.0) * p * p);
  }
}

std::vector<double> derivative_matrix(const std::vector<double>& x) {
  const int n = (int)x.size();
  std::vector<double> lam(n, 1.0), D(n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (x[j] - x[k]);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j)
      if (j != i) {
        D[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
        s += D[i * n + j];
      }
    D[i * n + i] = -s;
  }
  return D;
}

std::vector<double> lagrange(const std::vector<double>& xf, const std::vector<double>& t) {
  const int n = (int)xf.size(), m = (int)t.size();
  std::vector<double> lam(n, 1.0), L(m * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (xf[j] - xf[k]);
  for (int i = 0; i < m; ++i) {
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if (t[i] == xf[j]) hit = j;
    if (hit >= 0) { L[i * n + hit] = 1.0; continue; }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += lam[j] / (t[i] - xf[j]);
    for (int j = 0; j < n; ++j) L[i * n + j] = lam[j] / (t[i] - xf[j]) / den;
  }
  return L;
}

std::vector<double> radau_right(int M) {
  std::vector<double> tau;
  if (M == 1) { tau.push_back(1.0); return tau; }
  auto q = [M](double t) {
    double pm, dpm, pm1, dpm1;
    legendre_pd(M, t, pm, dpm);
    legendre_pd(M - 1, t, pm1, dpm1);
    return pm - pm1;
  };
  std::vector<double> in = roots(q, -1.0, 1.0, 4000);
  for (double t : in) tau.push_back(0.5 * (t + 1.0));
  tau.push_back(1.0);
  return tau;
}

static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  auto p = [n](double t) { double a, b; legendre_pd(n, t, a, b); return a; };
  x = roots(p, -1.0, 1.0, 4000);
  w.resize(x.size());
  for (size_t j = 0; j < x.size(); ++j) {
    double a, b;
    legendre_pd(n, x[j], a, b);
    w[j] = 2.0 / ((1.0 - x[j] * x[j]) * b * b);
  }
}

std::vector<double> nn_weights(const std::vector<double>& tau) {
  const int M = (int)tau.size();
  std::vector<double> xg, wg;
  gauss_legendre(M + 1, xg, wg);
  std::vector<double> W(M * M, 0.0);
  double lo = 0.0;
  for (int m = 0; m < M; ++m) {
    double hi = tau[m];
    std::vector<double> s(xg.size());
    for (size_t q = 0; q < xg.size(); ++q) s[q] = lo + (hi - lo) * 0.5 * (xg[q] + 1.0);
    std::vector<double> L = lagrange(tau, s);
    for (int i = 0; i < M; ++i) {
      double acc = 0.0;
      for (size_t q = 0; q < xg.size(); ++q) acc += wg[q] * L[q * M + i];
      W[m * M + i] = 0.5 * (hi - lo) * acc;
    }
    lo = hi;
  }
  return W;
}


std::vector<double> legendre_analysis(int P, const std::vector<double>& x, const std::vector<double>& w) {
  const int n = P + 1;
  std::vector<double> phi((size_t)n * n);  // phi[k*n + i] = phi_k(x_i)
  for (int i = 0; i < n; ++i) {
    double pm = 1.0, pk = x[i];
    for (int k = 0; k < n; ++k) {
      double val;
      if (k == 0) {
        val = 1.0;
      } else if (k == 1) {
        val = x[i];
      } else {
        const double next = ((2.0 * k - 1.0) * x[i] * pk - (k - 1.0) * pm) / k;
        pm = pk;
        pk = next;
        val = next;
      }
      phi[(size_t)k * n + i] = std::sqrt(0.5 * (2.0 * k + 1.0)) * val;
    }
  }
  std::vector<double> A((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    double g = 0.0;
    for (int j = 0; j < n; ++j) g += w[j] * phi[(size_t)k * n + j] * phi[(size_t)k * n + j];
    for (int i = 0; i < n; ++i) A[(size_t)k * n + i] = w[i] * phi[(size_t)k * n + i] / g;
  }
  return A;
}

void fds_axis(const std::vector<double>& w, const std::vector<double>& D, double rh, double pen,
              std::vector<double>& S, std::vector<double>& lam) {
  const int n = (int)w.size();
  std::vector<double> K((size_t)n * n, 0.0);
  // volume: D^T W D
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += D[k * n + i] * w[k] * D[k * n + j];
      K[i * n + j] = v;
    }
  // the element's own face terms at its two end nodes
  for (int side = 0; side < 2; ++side) {
    const int e = side ? n - 1 : 0;
    const double sgn = side ? 1.0 : -1.0;
    for (int j = 0; j < n; ++j) {
      K[j * n + e] -= 0.5 * sgn * D[e * n + j];  // D^T e e^T: row j, column e
      K[e * n + j] -= 0.5 * sgn * D[e * n + j];  // e e^T D: row e, column j
    }
    K[e * n + e] += 0.5 * pen;
  }
  for (double& v : K) v *= rh * rh;
  // B = W^-1/2 K W^-1/2, symmetric; cyclic Jacobi rotations B -> Q^T B Q
  std::vector<double> B((size_t)n * n), Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    Q[i * n + i] = 1.0;
    for (int j = 0; j < n; ++j) B[i * n + j] = K[i * n + j] / std::sqrt(w[i] * w[j]);
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) B[i * n + j] = B[j * n + i] = 0.5 * (B[i * n + j] + B[j * n + i]);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? diag : off) += B[i * n + j] * B[i * n + j];
    if (off <= 1e-32 * diag) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double bpq = B[p * n + q];
        if (bpq == 0.0) continue;
        const double theta = 0.5 * (B[q * n + q] - B[p * n + p]) / bpq;
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double bkp = B[k * n + p], bkq = B[k * n + q];
          B[k * n + p] = c * bkp - sn * bkq;
          B[k * n + q] = sn * bkp + c * bkq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double bpk = B[p * n + k], bqk = B[q * n + k];
          B[p * n + k] = c * bpk - sn * bqk;
          B[q * n + k] = sn * bpk + c * bqk;
        }
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - sn * qkq;
          Q[k * n + q] = sn * qkp + c * qkq;
        }
      }
  }
  S.assign((size_t)n * n, 0.0);
  lam.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    lam[k] = B[k * n + k];
    for (int i = 0; i < n; ++i) S[i * n + k] = Q[i * n + k] / std::sqrt(w[i]);
  }
}

}  // namespace sisdc

