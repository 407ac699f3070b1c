// Host-callable launchers of the HIP kernels (kernels.hip).  Each enqueues on
// stream s and returns the launch status; none synchronises.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace sisdc {

constexpr int kVecBlocks = 1024;  // grid cap of the grid-stride vector kernels

hipError_t launch_conv(const double* u, double* out, const Geo& g, const EqP& q, const double* tab,
                       hipStream_t s);
// trace pass + apply pass: out = alpha M x + beta K_D x; if dotv != NULL the
// dot product (out, dotv) is reduced into scal->pAp.  done (nullable): skip
// when *done != 0.
hipError_t launch_sipg(const double* x, double* out, int nv, const CoefP& cf, double* trace, double alpha,
                       double beta, double ctau, const Geo& g, const double* tab, const double* dotv,
                       double* partials, unsigned* counter, CGScal* scal, const int* done,
                       hipStream_t s);
hipError_t launch_helm_diag(double* diag, int nv, const CoefP& cf, double dtm, double ctau, const Geo& g,
                            const double* tab, hipStream_t s);
hipError_t launch_lincomb(double* out, const LinComb& lc, long n, const double* mw, int np, hipStream_t s);
hipError_t launch_cg_init(const double* b, const double* Ax, const double* diag, double* r, double* z,
                          double* p, long n, double* partials, unsigned* counter, CGScal* scal,
                          hipStream_t s);
hipError_t launch_cg_update(double* x, double* r, double* z, const double* p, const double* Ap,
                            const double* diag, long n, double* partials, unsigned* counter, CGScal* scal,
                            hipStream_t s);
hipError_t launch_cg_dir(double* p, const double* z, long n, const CGScal* scal, hipStream_t s);
hipError_t launch_space_transfer(const double* in, double* out, int nv, int dim, int n1i, int n1o, int E,
                                 const double* A, hipStream_t s);
hipError_t launch_euler_lam(const double* u, long vs, const EqP& q, int dim, double* partials,
                            unsigned* counter, double* result, hipStream_t s);
int elem_block_count(const Geo& g);

}  // namespace sisdc
