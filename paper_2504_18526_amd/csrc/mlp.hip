// Element-local MLP of the learned PCG initial guess: GEMMs on the matrix
// cores (FP32 MFMA for training, BF16 MFMA with FP32 accumulation for
// inference), fused bias + ReLU epilogues, the backward pass and Adam.
//
// Rows are (element, component) pairs: a nodal vector [var][elem][node] is
// already a row-major [rows x n] matrix with n = (P+1)^d.
//
// Network: z1 = W1 x + b1, a1 = relu(z1), z2 = W2 a1 + b2, a2 = relu(z2),
// y = W3 a2 + b3; flat parameters W1 (H x n), b1, W2 (H x H), b2, W3 (n x H),
// b3, row-major [out][in].
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"
#include "mlp.hpp"

namespace sisdc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[N]) (relu).  op(A)(i,k) =
// transA ? A[k*lda + i] : A[i*lda + k]; op(B)(k,j) = transB ? B[j*ldb + k] :
// B[k*ldb + j].  A workgroup of four waves computes a 64 x 64 tile of C, each
// wave a 32 x 32 quarter as 2 x 2 MFMA blocks of 16 x 16.  K advances in
// slabs of 32: the workgroup stages op(A) (64 x 32) and op(B)^T (64 x 32) in
// LDS, k contiguous, rounded to bfloat16 on the way in (BF16) or kept in
// FP32, and the waves read their operands from there.  Out-of-range
// operands are staged as 0 and out-of-range results are not stored.  BF16:
// FP32 accumulation.  VEC: op(A) and op(B)^T are k-contiguous in memory
// (transA = 0, transB = 1; K, lda and ldb multiples of 4, A and B 16-byte
// aligned, all checked at launch), so each thread stages four consecutive k
// per load and per LDS store.
//
// MFMA operand layout (lane l of 64, r = l % 16, q = l / 16):
//   16x16x32 bf16 (gfx950): A(row r, k 8q + t), B(k 8q + t, col r), t = 0..7;
//   16x16x4 f32: A(row r, k q), B(k q, col r);
//   result: lane l, register j holds row 4q + j, col r.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

template <bool BF16>
struct GemmTile {
  static constexpr int TM = 64, TN = 64, TK = BF16 ? 128 : 64;  // K slab: four (BF16) or sixteen (FP32) MFMA steps
  static constexpr int LD = BF16 ? TK + 8 : TK + 4;  // padded row (k) length; 16-byte aligned rows
  using E = typename std::conditional<BF16, short, float>::type;
};

template <bool BF16, bool VEC>
__global__ void __launch_bounds__(256, 4)
k_gemm(int M, int N, int K, const float* __restrict__ A, int lda, int transA, const float* __restrict__ B, int ldb,
       int transB, float* __restrict__ C, int ldc, const float* __restrict__ bias, int relu) {
  using G = GemmTile<BF16>;
  using E = typename G::E;
  constexpr int TM = G::TM, TN = G::TN, TK = G::TK, LD = G::LD;
  __shared__ __align__(16) E sA[TM * LD];  // sA[i*LD + k] = op(A)(i0 + i, k0 + k)
  __shared__ __align__(16) E sB[TN * LD];  // sB[j*LD + k] = op(B)(k0 + k, j0 + j)
  const int t = threadIdx.x, l = t & 63, wv = t >> 6;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  const int wi = (wv >> 1) * 32, wj = (wv & 1) * 32;
  const int r = l % 16, q = l / 16;
  floatx4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  auto put = [](float v) -> E {
    if constexpr (BF16) return to_bf16(v);
    else return v;
  };
  for (int k0 = 0; k0 < K; k0 += TK) {
    if constexpr (VEC) {
      // rows i of op(A) and of op(B)^T (TM = TN): four k per thread and step,
      // consecutive threads along k; K % 4 == 0, so a group is all in or all out
      constexpr int K4 = TK / 4;
#pragma unroll
      for (int st = 0; st < (TM * TK) / (4 * 256); ++st) {
        const int idx = t + 256 * st;
        const int i = idx / K4, k = 4 * (idx % K4), gk = k0 + k;
        float4 v = {0.f, 0.f, 0.f, 0.f}, u = {0.f, 0.f, 0.f, 0.f};
        if (i0 + i < M && gk < K) v = *reinterpret_cast<const float4*>(A + (long)(i0 + i) * lda + gk);
        if (j0 + i < N && gk < K) u = *reinterpret_cast<const float4*>(B + (long)(j0 + i) * ldb + gk);
        if constexpr (BF16) {
          auto cvt = [](float4 f) { return shortx4{to_bf16(f.x), to_bf16(f.y), to_bf16(f.z), to_bf16(f.w)}; };
          *reinterpret_cast<shortx4*>(&sA[i * LD + k]) = cvt(v);
          *reinterpret_cast<shortx4*>(&sB[i * LD + k]) = cvt(u);
        } else {
          *reinterpret_cast<float4*>(&sA[i * LD + k]) = v;
          *reinterpret_cast<float4*>(&sB[i * LD + k]) = u;
        }
      }
    } else {
      // stage: 2048 values of each operand, 8 per thread, consecutive threads
      // along the operand's contiguous global axis
#pragma unroll 8
      for (int st = 0; st < (TM * TK) / 256; ++st) {
        const int idx = t + 256 * st;
        int i, k;
        if (transA) {
          k = idx / TM;
          i = idx % TM;
        } else {
          i = idx / TK;
          k = idx % TK;
        }
        const int gi = i0 + i, gk = k0 + k;
        float v = 0.f;
        if (gi < M && gk < K) v = transA ? A[(long)gk * lda + gi] : A[(long)gi * lda + gk];
        sA[i * LD + k] = put(v);
        int j, kb;
        if (transB) {
          j = idx / TK;
          kb = idx % TK;
        } else {
          kb = idx / TN;
          j = idx % TN;
        }
        const int gj = j0 + j, gkb = k0 + kb;
        float u = 0.f;
        if (gj < N && gkb < K) u = transB ? B[(long)gj * ldb + gkb] : B[(long)gkb * ldb + gj];
        sB[j * LD + kb] = put(u);
      }
    }
    __syncthreads();
    if constexpr (BF16) {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 32) {
        bf16x8 av[2], bv[2];
        for (int a = 0; a < 2; ++a)
          av[a] = __builtin_bit_cast(bf16x8,
                                     *reinterpret_cast<const shortx8*>(&sA[(wi + 16 * a + r) * LD + kk + 8 * q]));
        for (int b = 0; b < 2; ++b)
          bv[b] = __builtin_bit_cast(bf16x8,
                                     *reinterpret_cast<const shortx8*>(&sB[(wj + 16 * b + r) * LD + kk + 8 * q]));
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        float av[2], bv[2];
        for (int a = 0; a < 2; ++a) av[a] = sA[(wi + 16 * a + r) * LD + kk + q];
        for (int b = 0; b < 2; ++b) bv[b] = sB[(wj + 16 * b + r) * LD + kk + q];
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();  // the next slab overwrites the tiles
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int jj = 0; jj < 4; ++jj) {
        const int i = i0 + wi + 16 * a + 4 * q + jj, j = j0 + wj + 16 * b + r;
        if (i < M && j < N) {
          float v = acc[a][b][jj];
          if (bias) v += bias[j];
          if (relu) v = fmaxf(v, 0.f);
          C[(long)i * ldc + j] = v;
        }
      }
}

// dY = (Y - T) / B; per-block partial sums of (Y - T)^2
__global__ void k_loss_grad(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY, long n,
                            float invB, double* part) {
  __shared__ double sred[16];
  double a = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = d * invB;
    a += (double)d * (double)d;
  }
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0) sred[wid] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sred[w];
    part[blockIdx.x] = s;
  }
}

// dZ = dA * (Z > 0)
__global__ void k_relu_back(const float* __restrict__ dA, const float* __restrict__ Z, float* __restrict__ dZ, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dZ[i] = Z[i] > 0.f ? dA[i] : 0.f;
}

// out[j] = sum over rows r (in order) of X[r * ld + j]
__global__ void k_colsum(const float* __restrict__ X, int rows, int cols, int ld, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += X[(long)r * ld + j];
  out[j] = s;
}

// Adam step k (1-based) on a flat parameter vector
__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Mass-scaled rows z = M^-1 r (mw: the n diagonal mass entries of an
// element), their norms |z| (FP64) and the normalised rows X = z / |z| (FP32).
// One wave per row.
__global__ void k_row_normalise(const double* __restrict__ r, int rows, int n, const double* __restrict__ mw,
                                float* __restrict__ X, double* __restrict__ nrm) {
  const int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const double* rr = r + (long)row * n;
  double s = 0.0;
  for (int k = lane; k < n; k += 64) {
    const double z = rr[k] / mw[k];
    s += z * z;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  const double nr = sqrt(s);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int k = lane; k < n; k += 64) X[(long)row * n + k] = (float)(rr[k] / mw[k] * inv);
  if (lane == 0) nrm[row] = nr;
}

// xnew = x + |z_row| * Y  (the network's correction, scaled back)
// the network's correction of every row: delta = |z0_row| Y_row
__global__ void k_guess_delta(const float* __restrict__ Y, const double* __restrict__ nrm, int rows, int n,
                              double* __restrict__ delta) {
  const long tot = (long)rows * n;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x)
    delta[i] = nrm[i / n] * (double)Y[i];
}

// x += alpha delta with the step that minimises the A-norm of the error
// along delta: alpha = (delta, r0) / (delta, A delta) from dots[0..1]; the
// error's A-norm then drops by (delta, r0)^2 / (delta, A delta).  A step
// that is not positive and finite is refused (counted in *rejected).
__global__ void k_guess_step(double* __restrict__ x, const double* __restrict__ delta, long n,
                             const double* __restrict__ dots, int* rejected) {
  const double alpha = dots[1] > 0.0 ? dots[0] / dots[1] : 0.0;
  const bool take = alpha > 0.0 && alpha < 1e300;
  if (blockIdx.x == 0 && threadIdx.x == 0 && !take) rejected[0] += 1;
  if (!take) return;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] += alpha * delta[i];
}

// harvest rows: X[row] = z0_row / |z0_row|, T[row] = (x - x0)_row / |z0_row|,
// z0 = M^-1 r0
__global__ void k_harvest(const double* __restrict__ r0, const double* __restrict__ x, const double* __restrict__ x0,
                          const double* __restrict__ nrm, int rows, int n, const double* __restrict__ mw,
                          float* __restrict__ X, float* __restrict__ T) {
  const long tot = (long)rows * n;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
    const double nr = nrm[i / n];
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    X[i] = (float)(r0[i] / mw[i % n] * inv);
    T[i] = (float)((x[i] - x0[i]) * inv);
  }
}

// ---------------------------------------------------------------- launchers
static inline int gblocks(long n) {
  long b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_gemm(int M, int N, int K, const float* A, int lda, int transA, const float* B, int ldb, int transB,
                       float* C, int ldc, const float* bias, int relu, int bf16, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  const bool vec = !transA && transB && K % 4 == 0 && lda % 4 == 0 && ldb % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(A) % 16 == 0 && reinterpret_cast<uintptr_t>(B) % 16 == 0;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, M, N, K, A, lda, transA, B, ldb, transB, C, ldc, bias, relu);
  };
  if (bf16)
    vec ? go(k_gemm<true, true>) : go(k_gemm<true, false>);
  else
    vec ? go(k_gemm<false, true>) : go(k_gemm<false, false>);
  return hipGetLastError();
}

// Forward pass of `rows` rows: Z1, A1, Z2, A2 (each rows x H) and Y (rows x n)
hipError_t mlp_forward(const MlpShape& sh, const float* theta, const float* X, int rows, float* Z1, float* A1,
                       float* Z2, float* A2, float* Y, int bf16, hipStream_t s) {
  const int n = sh.n, H = sh.H;
  const float *W1 = theta, *b1 = W1 + (long)H * n, *W2 = b1 + H, *b2 = W2 + (long)H * H, *W3 = b2 + H,
              *b3 = W3 + (long)n * H;
  hipError_t e;
  if (Z1) {
    if ((e = launch_gemm(rows, H, n, X, n, 0, W1, n, 1, Z1, H, b1, 0, bf16, s)) != hipSuccess) return e;
    if ((e = launch_gemm(rows, H, n, X, n, 0, W1, n, 1, A1, H, b1, 1, bf16, s)) != hipSuccess) return e;
    if ((e = launch_gemm(rows, H, H, A1, H, 0, W2, H, 1, Z2, H, b2, 0, bf16, s)) != hipSuccess) return e;
  } else {
    if ((e = launch_gemm(rows, H, n, X, n, 0, W1, n, 1, A1, H, b1, 1, bf16, s)) != hipSuccess) return e;
  }
  if ((e = launch_gemm(rows, H, H, A1, H, 0, W2, H, 1, A2, H, b2, 1, bf16, s)) != hipSuccess) return e;
  return launch_gemm(rows, n, H, A2, H, 0, W3, H, 1, Y, n, b3, 0, bf16, s);
}

// Loss partials, gradient into g (flat, same layout as theta); work buffers
// dY (rows x n), dA, dZ (rows x H).  FP32 throughout.
hipError_t mlp_backward(const MlpShape& sh, const float* theta, const float* X, const float* T, int rows,
                        const float* Z1, const float* A1, const float* Z2, const float* A2, const float* Y, float* dY,
                        float* dA, float* dZ, float* g, double* loss_part, hipStream_t s) {
  const int n = sh.n, H = sh.H;
  const float *W2 = theta + (long)H * n + H, *W3 = W2 + (long)H * H + H;
  float *dW1 = g, *db1 = dW1 + (long)H * n, *dW2 = db1 + H, *db2 = dW2 + (long)H * H, *dW3 = db2 + H,
        *db3 = dW3 + (long)n * H;
  const long ny = (long)rows * n, nh = (long)rows * H;
  hipLaunchKernelGGL(k_loss_grad, dim3(64), dim3(256), 0, s, Y, T, dY, ny, 1.f / rows, loss_part);
  hipError_t e;
  if ((e = launch_gemm(n, H, rows, dY, n, 1, A2, H, 0, dW3, H, nullptr, 0, 0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((n + 255) / 256), dim3(256), 0, s, dY, rows, n, n, db3);
  if ((e = launch_gemm(rows, H, n, dY, n, 0, W3, H, 0, dA, H, nullptr, 0, 0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_relu_back, dim3(gblocks(nh)), dim3(256), 0, s, dA, Z2, dZ, nh);
  if ((e = launch_gemm(H, H, rows, dZ, H, 1, A1, H, 0, dW2, H, nullptr, 0, 0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, dZ, rows, H, H, db2);
  if ((e = launch_gemm(rows, H, H, dZ, H, 0, W2, H, 0, dA, H, nullptr, 0, 0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_relu_back, dim3(gblocks(nh)), dim3(256), 0, s, dA, Z1, dZ, nh);
  if ((e = launch_gemm(H, n, rows, dZ, H, 1, X, n, 0, dW1, n, nullptr, 0, 0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, dZ, rows, H, H, db1);
  return hipGetLastError();
}

hipError_t launch_adam(float* th, float* m, float* v, const float* g, long n, float lr, int step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(gblocks(n)), dim3(256), 0, s, th, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_row_normalise(const double* r, int rows, int n, const double* mw, float* X, double* nrm,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_row_normalise, dim3((rows + 3) / 4), dim3(256), 0, s, r, rows, n, mw, X, nrm);
  return hipGetLastError();
}

hipError_t launch_guess_delta(const float* Y, const double* nrm, int rows, int n, double* delta, hipStream_t s) {
  hipLaunchKernelGGL(k_guess_delta, dim3(gblocks((long)rows * n)), dim3(256), 0, s, Y, nrm, rows, n, delta);
  return hipGetLastError();
}

hipError_t launch_guess_step(double* x, const double* delta, long n, const double* dots, int* rejected,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_guess_step, dim3(gblocks(n)), dim3(256), 0, s, x, delta, n, dots, rejected);
  return hipGetLastError();
}

hipError_t launch_harvest(const double* r0, const double* x, const double* x0, const double* nrm, int rows, int n,
                          const double* mw, float* X, float* T, hipStream_t s) {
  hipLaunchKernelGGL(k_harvest, dim3(gblocks((long)rows * n)), dim3(256), 0, s, r0, x, x0, nrm, rows, n, mw, X, T);
  return hipGetLastError();
}

}  // namespace sisdc
