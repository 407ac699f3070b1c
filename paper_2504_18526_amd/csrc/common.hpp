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
enum { EQ_CONVDIFF = 0, EQ_BURGERS = 1, EQ_EULER = 2, EQ_NS = 3 };
struct EqP {
  int eq, nv;
  double a[3];
  double nu;
  double gamma;
  double mu;     // dynamic viscosity (Navier-Stokes)
  double lam_T;  // heat conductivity mu c_p / Pr
  double R;      // gas constant
};

// Implicit coefficient D_ij = c w^2 v_i v_j + nu delta_ij, w = ub[node] or 1,
// in the arithmetic type T of the operator.
template <typename T>
struct CoefT {
  T c;
  T v[3];
  T nu;
  const T* ub;  // state the coefficient is evaluated at (nullable)
};
using CoefP = CoefT<double>;

// Result record of one CG solve, written by the single block that detects
// convergence (or by block 0 of every iteration kernel for the last state).
struct CGRes {
  double rr;      // squared residual norm at the last checked iterate
  double bb;      // squared norm of the right-hand side
  double thresh;  // rtol^2 * bb
  int it;         // iterations taken when converged
  int it_last;    // last iteration index that ran
};

// Device work buffers of the Chronopoulos-Gear PCG (one matvec and one
// fused reduction phase per iteration), in the arithmetic type T.
template <typename T>
struct CGStateT {
  T *x, *r, *z, *p, *s, *w;
  T* trace;        // face traces of (D grad z)
  const T* b;
  const T* diag;
  T* gam;          // 3 x cap partial sums of (r, z), by iteration mod 3
  T* rr;           // 2 x cap partial sums of (r, r), by iteration mod 2
  T* del;          // cap partial sums of (w, z)
  T* bbp;          // cap partial sums of (b, b)
  T* alpha;        // 2 step lengths, by iteration mod 2
  int* done_gen;   // id of the last solve that converged
  CGRes* res;
  T tol2;
  int cap;         // partial slots per array (>= grid of the element kernels)
};
using CGState = CGStateT<double>;

// Arguments of the persistent (one launch per solve) PCG kernel.  Face data
// exchanged between workgroups and the barrier records go through
// device-scope (L2 write-through) stores and loads; bar[64] is the abort word.
struct PCGArgs {
  const double* b;
  double* x;       // out: solution
  const double* x0;  // in: initial guess (may equal x)
  unsigned long long* fz;  // face values of the exchanged vector, 2 x [c][e][dim][side][f] x 2 tagged words
  unsigned long long* ft;  // face traces of (D grad .),      2 x [c][e][dim][side][f] x 2 tagged words
  unsigned long long* part;  // barrier records: 2 (barrier parity) x cap records of 16 tagged words
  unsigned* bar;
  CGRes* res;      // result record of this solve
  double tol2;
  double dtm;
  double ctau;
  int maxit;
  int cap;
  long spin_limit; // polls before a barrier gives up (abort, no hang)
  unsigned tag0;   // tag of the launch's first barrier; the launch uses tag0, tag0 + 1, ...,
                   // none of them in a record at launch time, and never 0
};

// Up to 8 vectors combined node-wise: out = sum_j c_j (m_j ? Jw : 1) x_j.
struct LinComb {
  const double* x[8];
  double c[8];
  int m[8];
  int n;
};

}  // namespace sisdc
