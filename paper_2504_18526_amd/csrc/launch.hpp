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

hipError_t launch_conv(const double* u, double* out, const Geo& g, const EqP& q, const double* tab,
                       hipStream_t s);
// face traces of (D grad x)
hipError_t launch_sipg_trace(const double* x, int nv, const CoefP& cf, double* trace, const Geo& g,
                             const double* tab, hipStream_t s);
// out = alpha M x + beta K_D x from the traces of x; part != NULL stores the
// block partials of (out, dotv); done_gen != NULL skips when *done_gen == id
hipError_t launch_sipg_apply(const double* x, double* out, int nv, const CoefP& cf, const double* trace,
                             double alpha, double beta, double ctau, const Geo& g, const double* tab,
                             const double* dotv, double* part, const int* done_gen, int id, hipStream_t s);
// trace pass + apply pass
hipError_t launch_sipg(const double* x, double* out, int nv, const CoefP& cf, double* trace, double alpha,
                       double beta, double ctau, const Geo& g, const double* tab, hipStream_t s);
hipError_t launch_helm_diag(double* diag, int nv, const CoefP& cf, double dtm, double ctau, const Geo& g,
                            const double* tab, hipStream_t s);
hipError_t launch_cg_start(const CGState& cg, int nv, const CoefP& cf, const Geo& g, const double* tab,
                           hipStream_t s);
hipError_t launch_cg_iter(const CGState& cg, int nv, const CoefP& cf, const Geo& g, const double* tab, int it,
                          int id, hipStream_t s);
hipError_t launch_lincomb(double* out, const LinComb& lc, long n, const double* mw, int np, hipStream_t s);
hipError_t launch_space_transfer(const double* in, double* out, int nv, int dim, int n1i, int n1o, int E,
                                 const double* A, hipStream_t s);
hipError_t launch_euler_lam(const double* u, long vs, const EqP& q, int dim, double* part, double* result,
                            hipStream_t s);
// Persistent PCG: one cooperative launch per solve (pcg_persistent.hip).
// Fails with hipErrorCooperativeLaunchTooLarge when the level's tiles exceed
// max_blocks (co-resident workgroups) or the partial-sum capacity.
hipError_t launch_pcg_persistent(const PCGArgs& a, int nv, const CoefP& cf, const Geo& g, const double* tab,
                                 int max_blocks, hipStream_t s);
int pcg_persistent_blocks_per_cu(const Geo& g, int nv);
int elem_tile_count(const Geo& g);
int reduce_grid(const Geo& g);

}  // namespace sisdc
