// Host-callable launchers of the HIP kernels (kernels.hip).  Each enqueues on
// stream s and returns the launch status; none synchronises.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"

namespace sisdc {

// grid cap of the element kernels that write partial sums (their consumers
// sum all partials in every block)
constexpr int kElemCap = 512;

// out = C(u) for `nodes` consecutive node vectors of u (each nv * E * np
// values) into the same number of consecutive vectors of out
hipError_t launch_conv(const double* u, double* out, const Geo& g, const EqP& q, const double* tab,
                       hipStream_t s, int nodes = 1);
// The SIPG and PCG launchers exist for double (FP64 path) and float (the
// inner solves of the mixed-precision path).
#define SISDC_DECLARE_PRECISION_LAUNCHERS(T)                                                                    \
  /* face traces of (D grad x) */                                                                               \
  hipError_t launch_sipg_trace(const T* x, int nv, const CoefT<T>& cf, T* trace, const Geo& g, const T* tab,     \
                               hipStream_t s);                                                                  \
  /* out = alpha M x + beta K_D x from the traces of x; part != NULL stores the block partials of (out, dotv); \
     done_gen != NULL skips when *done_gen == id */                                                             \
  hipError_t launch_sipg_apply(const T* x, T* out, int nv, const CoefT<T>& cf, const T* trace, T alpha, T beta, \
                               T ctau, const Geo& g, const T* tab, const T* dotv, T* part, const int* done_gen, \
                               int id, hipStream_t s);                                                          \
  /* trace pass + apply pass */                                                                                 \
  hipError_t launch_sipg(const T* x, T* out, int nv, const CoefT<T>& cf, T* trace, T alpha, T beta, T ctau,     \
                         const Geo& g, const T* tab, hipStream_t s);                                            \
  hipError_t launch_helm_diag(T* diag, int nv, const CoefT<T>& cf, T dtm, T ctau, const Geo& g, const T* tab,    \
                              hipStream_t s);                                                                   \
  /* diag[0, NP) = the diagonal of M + dtm K_D on the first element of component 0 only (an isotropic level:   \
     the same on every element and component), then idg = 1 / diag there */                                     \
  hipError_t launch_iso_inv_diag(T* diag, T* idg, const CoefT<T>& cf, T dtm, T ctau, const Geo& g, const T* tab, \
                                 hipStream_t s);                                                                \
  hipError_t launch_cg_start(const CGStateT<T>& cg, int nv, const CoefT<T>& cf, const Geo& g, const T* tab,     \
                             hipStream_t s);                                                                    \
  hipError_t launch_cg_iter(const CGStateT<T>& cg, int nv, const CoefT<T>& cf, const Geo& g, const T* tab,      \
                            int it, int id, hipStream_t s);                                                     \
  /* Isotropic hexahedral path (D = nu I constant on the level, dim 3, P in {1, 3, 7}): the matvec computes    \
     the neighbours' face fluxes itself (no trace pass) and may scale its operand node by node by isc (NP       \
     values); the streaming CG kernels never store z = r idg (idg: NP-periodic inverse Jacobi diagonal). */      \
  bool sipg_iso_path(const Geo& g, const CoefT<T>& cf);                                                         \
  hipError_t launch_sipg_apply_iso(const T* x, const T* isc, T* out, int nv, const CoefT<T>& cf, T alpha,       \
                                   T beta, T ctau, const Geo& g, const T* tab, T* part, const int* done_gen,    \
                                   int id, hipStream_t s);                                                      \
  /* cg.b == NULL: the right-hand side is the combination bl (FP64 only; mw the element's mass weights) */     \
  hipError_t launch_cg_start_iso(const CGStateT<T>& cg, const T* idg, int nv, const Geo& g, const LinComb* bl,   \
                                 const double* mw, hipStream_t s);                                              \
  hipError_t launch_cg_iter_iso(const CGStateT<T>& cg, const T* idg, int nv, const Geo& g, int it, int id,      \
                                hipStream_t s);                                                                 \
  /* the streaming CG updates x every second iteration; this adds the step still pending after its loop */     \
  hipError_t launch_cg_fix_iso(const CGStateT<T>& cg, long n, int id, hipStream_t s);

// z = A_ee^-1 r per element: the element-block Jacobi preconditioner of the
// isotropic operator M + dtk K_{I} by fast diagonalisation (fds: the S and
// lam tables of the three axes, fds_axis); with part_rz != NULL also the
// block partials of (r, z) and (r, r) in the streaming CG's grid.
hipError_t launch_fds(const double* r, double* z, int nv, const Geo& g, const double* fds, double dtk,
                      double* part_rz, double* part_rr, const int* done_gen, int id, hipStream_t s);

// grid of the streaming isotropic CG's start and update kernels (their
// partial-sum count) on a level; 0 where that path does not apply
int iso_cg_grid(const Geo& g);

SISDC_DECLARE_PRECISION_LAUNCHERS(double)
SISDC_DECLARE_PRECISION_LAUNCHERS(float)

// out = add + V(u), the BR1 viscous term of Navier-Stokes (trace pass + apply
// pass); add == out (or NULL) accumulates onto out in place
hipError_t launch_visc(const double* u, const double* add, double* out, double* trace, const Geo& g, const EqP& q,
                       const double* tab, hipStream_t s);
hipError_t launch_lincomb(double* out, const LinComb& lc, long n, const double* mw, int np, hipStream_t s);
// out = add + alpha M x + beta K_{nu I} x on quadrilaterals with isotropic
// constant D (the 2-D isotropic matvec with an added vector; add must not
// overlap out); hipErrorInvalidValue where that kernel does not apply.
hipError_t launch_sipg_iso2_add(const double* x, const double* add, double* out, int nv, const CoefT<double>& cf,
                                double alpha, double beta, double ctau, const Geo& g, const double* tab,
                                hipStream_t s);
// out[o * n + i] = sum_j lc.c[o][j] lc.x[j][i], o < lc.nout, j < lc.nin (<= 8 each).
hipError_t launch_lincomb_multi(double* out, const LinCombMulti& lc, long n, hipStream_t s);
// 2:1 h-coarsening transfer between a fine level and the coarse level of
// nc[0] x nc[1] (x nc[2]) elements; mode 0: fine -> coarse with A (n1c x 2 n1f),
// mode 1: coarse -> fine with A (2 n1f x n1c).  hipErrorInvalidValue when a
// pair of fine elements does not fit the kernel's grid ((2 n1f)^dim > 2744).
hipError_t launch_space_transfer_h(const double* in, double* out, int nv, int dim, int n1f, int n1c, const int* nc,
                                   const double* A, int mode, hipStream_t s);
hipError_t launch_space_transfer(const double* in, double* out, int nv, int dim, int n1i, int n1o, int E,
                                 const double* A, hipStream_t s);
// The collocation residual of a level (all M nodes) in one pass; mw holds the
// np diagonal mass weights of one element. M outside 1..8 returns
// hipErrorInvalidValue before any launch.
hipError_t launch_colloc_residual(const CollocResid& c, long n, const double* mw, int np, hipStream_t s);
// y[o] = [y[o] +] X(sum_j c[o][j] x[j]) for o < t.nout, X the map A per
// direction; the two levels have the same E elements. Invalid counts return
// hipErrorInvalidValue before any launch.
hipError_t launch_space_time_transfer(const TransferMulti& t, int nv, int dim, int n1i, int n1o, int E,
                                      const double* A, hipStream_t s);
// mixed precision: FP64 -> FP32 copy; r32 = b - Ax with (r,r), (b,b) summed
// into tot[0..1] (FP64); x += e
// Persson-Peraire artificial viscosity per element from the state u (nv
// components, component 0 sensed): A the (P+1)^2 discrete Legendre
// transform, kappa the switch half-width kappa_s, c_s the scale of
// eps_0 = c_s (min_d h_d / P) lam_e.
hipError_t launch_av_sensor(const double* u, int nv, const Geo& g, const EqP& q, const double* A, double kappa,
                            double c_s, double* eps, hipStream_t s);
hipError_t launch_copy(const double* in, double* out, long n, hipStream_t s);
hipError_t launch_cast_f(const double* in, float* out, long n, hipStream_t s);
hipError_t launch_resid_cast(const double* b, const double* Ax, float* r32, long n, double* part, double* tot,
                             hipStream_t s);
hipError_t launch_add_f2d(double* x, const float* e, long n, hipStream_t s);
// Conservation correction after an implicit solve: x_c += (1^T b_c - 1^T M
// x_c) / mass_total for every component c (b a vector, or the combination lc
// when b is NULL); part holds at least 2 nv partials per block (part_cap
// values in all).  Two launches, deterministic fixed-order sums.
hipError_t launch_conserve(const double* b, const LinComb* lc, double* x, int nv, long vs, const double* mw, int np,
                           double mass_total, double* part, int part_cap, hipStream_t s);
// tot[0] = (a, b), tot[1] = (a, c) (deterministic partial sums in part)
hipError_t launch_dot2(const double* a, const double* b, const double* c, long n, double* part, double* tot,
                       hipStream_t s);
// result[0] = max over nodes of max_d (|v_d| + c), result[1] = min rho
hipError_t launch_euler_lam(const double* u, long vs, const EqP& q, int dim, double* part, double* result,
                            hipStream_t s);
// Persistent PCG: one launch per solve (pcg_persistent.hip), for scalar
// equations (nv = 1; hipErrorInvalidValue otherwise).  `cooperative`: through
// the cooperative-launch API; otherwise an ordinary launch, and the caller
// makes sure no other grid that waits across workgroups shares the device
// (all max_blocks workgroups are then resident together).  Fails with
// hipErrorCooperativeLaunchTooLarge when the level's tiles exceed max_blocks
// (co-resident workgroups) or the partial-sum capacity.
hipError_t launch_pcg_persistent(const PCGArgs& a, int nv, const CoefP& cf, const Geo& g, const double* tab,
                                 int max_blocks, bool cooperative, hipStream_t s);
int pcg_persistent_blocks_per_cu(const Geo& g, int nv);
int pcg_persistent_grid(const Geo& g);
int elem_tile_count(const Geo& g);
int reduce_grid(const Geo& g);

}  // namespace sisdc
