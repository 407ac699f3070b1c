// Plain-data descriptors shared by the host orchestration and the kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace sisdc {

constexpr int kMaxP = 8;

// Periodic uniform Cartesian mesh of one level.
struct Geo {
  int dim, P, n1, np, nf;  // n1 = P+1, np = n1^dim nodes, nf = n1^(dim-1) face nodes
  int ne[3];               // elements per axis
  int E;                   // total elements
  double h[3];             // element size per axis
  double rh2[3];           // 2 / h
  double J;                // prod h / 2
};

// Equation parameters.
enum { EQ_CONVDIFF = 0, EQ_BURGERS = 1, EQ_EULER = 2 };
struct EqP {
  int eq, nv;
  double a[3];
  double nu;
  double gamma;
};

// Implicit coefficient D_ij = c w^2 v_i v_j + nu delta_ij, w = ub[node] or 1.
struct CoefP {
  double c;
  double v[3];
  double nu;
  const double* ub;  // state the coefficient is evaluated at (nullable)
};

// Device-resident CG scalars.
struct CGScal {
  double rz, pAp, rr, bb, beta, tol2;
  int done, it, maxit, pad;
};

// Up to 8 vectors combined node-wise: out = sum_j c_j (m_j ? Jw : 1) x_j.
struct LinComb {
  const double* x[8];
  double c[8];
  int m[8];
  int n;
};

}  // namespace sisdc
