// Plain-data descriptors shared by the host orchestration and the kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace sisdc {

constexpr int kMaxP = 8;
constexpr int kMaxComp = 5;  // conserved components (Navier-Stokes in 3-D)

// Periodic uniform Cartesian mesh of one level.
struct Geo {
  int dim, P, n1, np, nf;  // n1 = P+1, np = n1^dim nodes, nf = n1^(dim-1) face nodes
  int ne[3];               // elements per axis
  int E;                   // total elements
  double h[3];             // element size per axis
  double rh2[3];           // 2 / h
  double J;                // prod h / 2
  int wl;                  // elements of one instance along the last axis (ensembles stack instances there)
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

// Implicit coefficient D_ij = c w^2 v_i v_j + (nu + eps_e) delta_ij,
// w = ub[node] or 1, eps_e the artificial viscosity of the node's element
// (0 without), in the arithmetic type T of the operator.
template <typename T>
struct CoefT {
  T c;
  T v[3];
  T nu;
  const T* ub;   // state the coefficient is evaluated at (nullable)
  const T* eps;  // artificial viscosity per element (nullable)
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
  const T* zs;     // streaming isotropic path with the block-Jacobi preconditioner: the stored z
                   // (its kernel writes z and the (r, z), (r, r) partials after every update); NULL: z = r idg
  const T* x0;     // streaming isotropic path: the initial guess when x does not hold it (else NULL);
                   // the first update of x reads it, so no copy x0 -> x precedes the solve
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
  // Conservation correction fused into the streaming isotropic PCG (NULL:
  // off).  Block partial sums by component c < kMaxComp, cap slots each:
  // cons[c cap, ...) sum b, cons[(5 + c) cap, ...) sum A x0 (= sum M x0),
  // cons[(10 + c) cap, ...) each update block's running sum over the
  // iterations k of alpha_k sum s_k (s_k = A p_k, so sum s_k = sum M p_k).
  // The last kernel shifts every component of x by (sum b - sum M x) /
  // mass_total, sum M x = sum M x0 + sum_k alpha_k sum M p_k.
  T* cons;
  long vs;         // values per component
  int nv;          // components (at most kMaxComp)
  int nparts;      // grid of the start and update kernels
  T mass_total;    // 1^T M 1 of one component
};
using CGState = CGStateT<double>;

// Arguments of the persistent (one launch per solve) PCG kernel.  Face data
// exchanged between workgroups and the barrier records go through
// device-scope (L2 write-through) stores and loads; bar[64] is the abort word.
// Up to 8 vectors combined node-wise: out = sum_j c_j (m_j ? Jw : 1) x_j.
struct LinComb {
  const double* x[8];
  double c[8];
  int m[8];
  int n;
};

// Up to 8 outputs from the same up to 8 vectors, node-wise:
// out[o] = sum_j c[o][j] x_j, each output vlen apart from the previous.
struct LinCombMulti {
  const double* x[8];
  double c[8][8];
  int nin, nout;
};

// The collocation residual of a level in one launch, for m = 1..M:
// out[m-1] = [g[m-1] +] sign (mw (u_m - u_{m-1}) - sum_i S[m-1][i] f[i]),
// u holding M+1 node vectors, f, g and out M, each vlen apart.
struct CollocResid {
  const double* u;
  const double* f;
  const double* g;  // or null
  double* out;
  double S[8][8];
  int M;
  double sign;
};

// A space-time transfer in one launch: for output node o < nout,
// y[o] = [y[o] +] X(sum_j c[o][j] x[j]), X the tensor-product space map of
// one element; y2[o], when set, receives the same values.
constexpr int kTransferIn = 16, kTransferOut = 8;
struct TransferMulti {
  const double* x[kTransferIn];
  double c[kTransferOut][kTransferIn];
  double* y[kTransferOut];
  double* y2[kTransferOut];
  int nin, nout, accumulate;
};

struct PCGArgs {
  const double* b;  // right-hand side, or null: then b = bl at every node
  LinComb bl;       // the right-hand side as a combination of vectors (used when b is null)
  const double* mw; // mass weights J w of one element's nodes (for bl's mass terms)
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

// A value moved across lanes by a DPP control (32-bit pieces); lanes whose
// source lies outside the pattern receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}

// Sum over the 64 lanes of a wave, in lane 63 (the other lanes hold partial
// sums): shifts by 1, 2, 4, 8 within each row of 16 lanes, then the row
// broadcasts of lanes 15 and 31.  Register-to-register (DPP), no LDS; the
// order of the additions is fixed, so every wave rounds alike.  Every lane
// of the wave must be active.
template <typename T>
__device__ __forceinline__ T wave_sum63(T x) {
  x += dpp_move<0x111, 0xf>(x);  // row_shr:1
  x += dpp_move<0x112, 0xf>(x);  // row_shr:2
  x += dpp_move<0x114, 0xf>(x);  // row_shr:4
  x += dpp_move<0x118, 0xf>(x);  // row_shr:8
  x += dpp_move<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_move<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

}  // namespace sisdc
