// Launchers of the learned-guess MLP kernels (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace sisdc {

struct MlpShape {
  int n;  // nodes per element row, (P+1)^d
  int H;  // hidden width
  long params() const { return (long)H * n + H + (long)H * H + H + (long)n * H + n; }
};

hipError_t launch_gemm(int M, int N, int K, const float* A, int lda, int transA, const float* B, int ldb, int transB,
                       float* C, int ldc, const float* bias, int relu, int bf16, hipStream_t s);
// Z1 == NULL: inference (only A1, A2, Y are written)
hipError_t mlp_forward(const MlpShape& sh, const float* theta, const float* X, int rows, float* Z1, float* A1,
                       float* Z2, float* A2, float* Y, int bf16, hipStream_t s);
hipError_t mlp_backward(const MlpShape& sh, const float* theta, const float* X, const float* T, int rows,
                        const float* Z1, const float* A1, const float* Z2, const float* A2, const float* Y, float* dY,
                        float* dA, float* dZ, float* g, double* loss_part, hipStream_t s);
hipError_t launch_adam(float* th, float* m, float* v, const float* g, long n, float lr, int step, hipStream_t s);
// z = M^-1 r per row (mw: the element's diagonal mass), |z| and z / |z|
hipError_t launch_row_normalise(const double* r, int rows, int n, const double* mw, float* X, double* nrm,
                                hipStream_t s);
// delta = |z0_row| Y_row; x += alpha delta, alpha = dots[0] / dots[1] =
// (delta, r0) / (delta, A delta) when positive (else refused, counted)
hipError_t launch_guess_delta(const float* Y, const double* nrm, int rows, int n, double* delta, hipStream_t s);
hipError_t launch_guess_step(double* x, const double* delta, long n, const double* dots, int* rejected,
                             hipStream_t s);
hipError_t launch_harvest(const double* r0, const double* x, const double* x0, const double* nrm, int rows, int n,
                          const double* mw, float* X, float* T, hipStream_t s);

}  // namespace sisdc
