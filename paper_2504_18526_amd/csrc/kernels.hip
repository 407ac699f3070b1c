// HIP kernels of the SI-MLSDC / DG-SEM hot path for gfx950 (MI355X).
//
// Element kernels: one workgroup holds EPB elements ("a tile"), one thread
// per node; the (P+1)^d nodal tile of each element and the 1-D GLL tables
// are staged in LDS, derivatives are sum-factorised (one 1-D contraction per
// axis).  Face terms read the neighbour's face trace straight from global
// memory (the neighbour index follows from the periodic Cartesian
// numbering).  Kernels that reduce are launched on at most kElemCap blocks
// and loop over tiles, so the number of partial sums stays small.
//
// Reductions never synchronise workgroups inside a kernel (a device-scope
// fence costs an L2 write-back on this multi-XCD part): every block writes
// one partial per quantity, and the consumer -- always a later kernel --
// sums all partials in a fixed order in every block.  Dot products are
// therefore deterministic, and no atomics are used.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "common.hpp"
#include "launch.hpp"
#include "gll_const.hpp"
#include "xcd.hpp"

namespace sisdc {

template <int DIM, int P>
struct EL {
  static constexpr int N1 = P + 1;
  static constexpr int NP = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
  static constexpr int NF = DIM == 2 ? N1 : N1 * N1;
  static constexpr int EPB = NP >= 256 ? 1 : 256 / NP;
  static constexpr int NT = ((EPB * NP + 63) / 64) * 64;
  // threads of the kernels with face tasks (a thread per node and a thread
  // per face node of the workgroup's elements, whichever needs more)
  static constexpr int NFT = EPB * 2 * DIM * NF;
  static constexpr int NTF = NT > NFT ? NT : ((NFT + 63) / 64) * 64;
  static constexpr int stride(int d) { return d == 0 ? 1 : (d == 1 ? N1 : N1 * N1); }
};

template <int DIM, int N1>
__device__ __forceinline__ void decomp(int n, int (&i)[3]) {
  i[0] = n % N1;
  i[1] = (n / N1) % N1;
  i[2] = DIM == 3 ? n / (N1 * N1) : 0;
}

template <int DIM, int N1>
__device__ __forceinline__ int face_index(int d, const int (&i)[3]) {
  if (DIM == 2) return i[1 - d];
  return d == 0 ? i[1] + N1 * i[2] : (d == 1 ? i[0] + N1 * i[2] : i[0] + N1 * i[1]);
}

// Element across the face of element e normal to d on side s (-1 / +1);
// periodic, along the last axis within the instance's block of g.wl
// elements.
__device__ __forceinline__ int neighbour(const Geo& g, int e, int d, int s) {
  int c[3];
  c[0] = e % g.ne[0];
  c[1] = (e / g.ne[0]) % g.ne[1];
  c[2] = g.dim == 3 ? e / (g.ne[0] * g.ne[1]) : 0;
  const int span = d == g.dim - 1 ? g.wl : g.ne[d];
  const int base = c[d] - c[d] % span;
  int loc = c[d] - base + s;
  if (loc < 0) loc += span;
  if (loc >= span) loc -= span;
  c[d] = base + loc;
  return c[0] + g.ne[0] * (c[1] + g.ne[1] * c[2]);
}

// ---------------------------------------------------------------- reductions

// Block-wide sums of K per-thread values; thread 0 stores them in
// part[k][blockIdx.x].  Every thread of the block must call it.
template <typename T, int K>
__device__ void block_partials(const T (&v)[K], T* const (&part)[K]) {
  __shared__ T sred[K][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    const T x = wave_sum63(v[k]);
    if (lane == 63) sred[k][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < K; ++k) {
      T s = T(0);
      for (int w = 0; w < nw; ++w) s += sred[k][w];
      part[k][blockIdx.x] = s;
    }
  }
}

// Block-wide sums of K per-thread values, returned to thread 0 (tot is
// undefined in the other threads).  Every thread of the block must call it.
template <typename T, int K>
__device__ void block_sum(const T (&v)[K], T (&tot)[K]) {
  __shared__ T sred[K][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    const T x = wave_sum63(v[k]);
    if (lane == 63) sred[k][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) {
      T s = T(0);
      for (int w = 0; w < nw; ++w) s += sred[k][w];
      tot[k] = s;
    }
}

// Fixed-order sums of the first n partials of each of K arrays, returned to
// every thread of the block (the same bits in every block).  Every thread of
// the block must call it.
template <typename T, int K>
__device__ void sum_partials(const T* const (&part)[K], int n, T (&tot)[K]) {
  __shared__ T sred[K][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    T a = T(0);
    for (int b = threadIdx.x; b < n; b += blockDim.x) a += part[k][b];
    a = wave_sum63(a);
    if (lane == 63) sred[k][wid] = a;
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    T s = T(0);
    for (int w = 0; w < nw; ++w) s += sred[k][w];
    tot[k] = s;
  }
  __syncthreads();
}

// f(std::integral_constant<int, 0>) ... f(std::integral_constant<int, N-1>):
// loop indices that are constant expressions.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------- fluxes
template <int NV>
__device__ __forceinline__ void flux(const EqP& q, int d, const double (&u)[NV], double (&f)[NV]) {
  if constexpr (NV == 1) {
    f[0] = q.eq == EQ_CONVDIFF ? q.a[d] * u[0] : 0.5 * u[0] * u[0];
  } else {
    constexpr int D = NV - 2;
    const double ir = 1.0 / u[0];
    double ke = 0.0;
    for (int k = 0; k < D; ++k) ke += u[1 + k] * u[1 + k];
    const double p = (q.gamma - 1.0) * (u[D + 1] - 0.5 * ke * ir);
    const double vd = u[1 + d] * ir;
    f[0] = u[1 + d];
    for (int k = 0; k < D; ++k) f[1 + k] = u[1 + k] * vd + (k == d ? p : 0.0);
    f[D + 1] = (u[D + 1] + p) * vd;
  }
}

template <int NV>
__device__ __forceinline__ double wave_speed(const EqP& q, int d, const double (&u)[NV]) {
  if constexpr (NV == 1) {
    return q.eq == EQ_CONVDIFF ? fabs(q.a[d]) : fabs(u[0]);
  } else {
    constexpr int D = NV - 2;
    const double ir = 1.0 / u[0];
    double ke = 0.0;
    for (int k = 0; k < D; ++k) ke += u[1 + k] * u[1 + k];
    const double p = (q.gamma - 1.0) * (u[D + 1] - 0.5 * ke * ir);
    return fabs(u[1 + d] * ir) + sqrt(q.gamma * p * ir);
  }
}

// ---------------------------------------------------------------- C(u)
// Node (i0, i1, i2) of face node fn on the face normal to d at index `at`
// along d (the inverse of face_index).
template <int DIM, int N1>
__device__ __forceinline__ int face_node(int d, int fn, int at) {
  if (DIM == 2) return d == 0 ? at + N1 * fn : fn + N1 * at;
  const int f0 = fn % N1, f1 = fn / N1;
  return d == 0 ? at + N1 * (f0 + N1 * f1) : (d == 1 ? f0 + N1 * (at + N1 * f1) : f0 + N1 * (f1 + N1 * at));
}

// The 2 DIM face neighbours of the workgroup's EPB elements e0 + l, in
// snb[l][2 d + side] (side 0: minus, 1: plus); every thread calls it.
template <int DIM, int EPB>
__device__ __forceinline__ void face_neighbours(const Geo& g, int e0, int* snb) {
  const int t = threadIdx.x;
  if (t < EPB * 2 * DIM) {
    const int l = t / (2 * DIM), f = t - l * 2 * DIM;
    snb[t] = e0 + l < g.E ? neighbour(g, e0 + l, f >> 1, (f & 1) ? 1 : -1) : 0;
  }
}

// out = C(u): -J w (sum_d 2/h_d D_d f_d(u)) - sum_faces J_f w_f (f* - f(u^-)).n
// A thread per node forms the volume term.  The face term is formed by a
// thread per face node (face and node are what every lane of a wave works
// on, so no wave runs a face at a fraction of its lanes) into LDS, and the
// node threads subtract it; the neighbours of the workgroup's elements are
// found once.
template <int DIM, int P, int NV>
__global__ void __launch_bounds__((EL<DIM, P>::NTF), 6)
k_conv(const double* __restrict__ u, double* __restrict__ out, Geo g, EqP q,
       const double* __restrict__ tab, long vs) {
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, NF = L::NF, EPB = L::EPB, NFC = 2 * DIM;
  __shared__ double sD[N1 * N1], sw[N1];
  __shared__ double sf[EPB * NV * NP];
  __shared__ double sF[EPB * NFC * NF * NV];
  __shared__ int snb[EPB * NFC];
  u += (long)blockIdx.y * NV * vs;  // node blockIdx.y of a batch of node vectors
  out += (long)blockIdx.y * NV * vs;
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB, e = e0 + le;
  const bool act = (le < EPB) && (e < g.E);
  static_assert(L::NT >= N1 * N1, "a thread per entry of the tables");
  // every global load of the prologue is issued before the first wait
  double uu[NV], acc[NV];
  for (int v = 0; v < NV; ++v) uu[v] = act ? u[v * vs + (long)e * NP + n] : 1.0;
  const double dv = t < N1 * N1 ? tab[t] : 0.0, wv = t < N1 ? tab[N1 * N1 + t] : 0.0;
  face_neighbours<DIM, EPB>(g, e0, snb);
  if (t < N1 * N1) sD[t] = dv;
  if (t < N1) sw[t] = wv;
  int ii[3];
  decomp<DIM, N1>(n, ii);
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  __syncthreads();
  // face tasks, a thread per (element, face, face node): the neighbour's
  // state at the face node of task k
  constexpr int NTASK = EPB * NFC * NF;
  auto outside = [&](int k, double (&uo)[NV]) {
    const int l = k / (NFC * NF), f = (k / NF) % NFC, fn = k % NF;
    const int nn = face_node<DIM, N1>(f >> 1, fn, (f & 1) ? 0 : P);
    const long nb = snb[l * NFC + f];
    for (int v = 0; v < NV; ++v) uo[v] = u[v * vs + nb * NP + nn];
  };
  // the first task's values are requested before the volume term and used
  // after it
  double uo0[NV];
  if (t < NTASK && e0 + t / (NFC * NF) < g.E) outside(t, uo0);
  for (int d = 0; d < DIM; ++d) {
    if (act) {
      double f[NV];
      flux<NV>(q, d, uu, f);
      for (int v = 0; v < NV; ++v) sf[(le * NV + v) * NP + n] = f[v];
    }
    __syncthreads();
    if (act) {
      const int st = L::stride(d);
      const int base = n - ii[d] * st;
      for (int v = 0; v < NV; ++v) {
        const double* row = &sf[(le * NV + v) * NP + base];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < N1; ++k) s += sD[ii[d] * N1 + k] * row[k * st];
        acc[v] -= g.rh2[d] * s;
      }
    }
    __syncthreads();
  }
  // the face terms into sF; the axis is made a constant, so the state's
  // components stay in registers
  for (int k = t; k < NTASK; k += L::NTF) {
    const int l = k / (NFC * NF), f = (k / NF) % NFC, fn = k % NF;
    if (e0 + l >= g.E) continue;
    double uo[NV];
    if (k == t)
      for (int v = 0; v < NV; ++v) uo[v] = uo0[v];
    else
      outside(k, uo);
    static_for<DIM>([&](auto dc) {
      constexpr int d = decltype(dc)::value;
      if ((f >> 1) != d) return;
      const int side = f & 1;
      const double sgn = side ? 1.0 : -1.0;
      const int nown = face_node<DIM, N1>(d, fn, side ? P : 0);
      double ui[NV], fi[NV], fo[NV];
      for (int v = 0; v < NV; ++v) ui[v] = u[v * vs + (long)(e0 + l) * NP + nown];  // in L2 (read by this workgroup)
      flux<NV>(q, d, ui, fi);
      flux<NV>(q, d, uo, fo);
      const double lam = fmax(wave_speed<NV>(q, d, ui), wave_speed<NV>(q, d, uo));
      // the face weight: w over the axes other than d
      const double wf = DIM == 2 ? sw[fn] : sw[fn % N1] * sw[fn / N1];
      const double jfwf = g.J * g.rh2[d] * wf;
      for (int v = 0; v < NV; ++v) {
        const double fin = sgn * fi[v], fout = sgn * fo[v];
        const double fstar = 0.5 * (fin + fout) - 0.5 * lam * (uo[v] - ui[v]);
        sF[k * NV + v] = jfwf * (fstar - fin);
      }
    });
  }
  __syncthreads();
  if (!act) return;
  double wn = 1.0;
  for (int d = 0; d < DIM; ++d) wn *= sw[ii[d]];
  for (int v = 0; v < NV; ++v) acc[v] *= g.J * wn;
  for (int d = 0; d < DIM; ++d)
    for (int side = 0; side < 2; ++side) {
      if (ii[d] != (side ? P : 0)) continue;
      const double* c = &sF[((le * NFC + 2 * d + side) * NF + face_index<DIM, N1>(d, ii)) * NV];
      for (int v = 0; v < NV; ++v) acc[v] -= c[v];
    }
  for (int v = 0; v < NV; ++v) out[v * vs + (long)e * NP + n] = acc[v];
}

// ---------------------------------------------------------------- viscous (NS)
// q = (v_1, ..., v_D, T) of a conservative state
template <int DIM>
__device__ __forceinline__ void prim_q(const EqP& q, const double (&u)[DIM + 2], double (&out)[DIM + 1]) {
  const double ir = 1.0 / u[0];
  double ke = 0.0;
  for (int k = 0; k < DIM; ++k) {
    out[k] = u[1 + k] * ir;
    ke += u[1 + k] * out[k];
  }
  const double p = (q.gamma - 1.0) * (u[DIM + 1] - 0.5 * ke);
  out[DIM] = p * ir / q.R;
}

// viscous flux in direction d from the state and the gradients G[e][j] = dq_j/dx_e
template <int DIM>
__device__ __forceinline__ void visc_flux(const EqP& q, int d, const double (&u)[DIM + 2],
                                          const double (&G)[DIM][DIM + 1], double (&f)[DIM + 2]) {
  const double ir = 1.0 / u[0];
  double div = 0.0;
  for (int k = 0; k < DIM; ++k) div += G[k][k];
  f[0] = 0.0;
  double work = 0.0;
  for (int i = 0; i < DIM; ++i) {
    const double tau = q.mu * (G[i][d] + G[d][i]) - (i == d ? 2.0 / 3.0 * q.mu * div : 0.0);
    f[1 + i] = tau;
    work += u[1 + i] * ir * tau;
  }
  f[DIM + 1] = work + q.lam_T * G[d][DIM];
}

// The viscous term in two passes over u, both built the same way as C(u):
// every global load of a pass is issued at its start (a face task's
// neighbour values included), and work on faces runs as face tasks, a
// thread per (element, face, face node), into LDS.
//
// BR1 lifted gradients at node n (indices ii) of element slot l: grad q from
// the LDS tiles sq (component j at sq[j * EPB * NP]) plus, at face nodes,
// (2/h_d) / w_face * ({q} - q^-) n_d = (2/h_d) / w_face * (q^+ - q^-) / 2 n_d
// with the jumps q^+ - q^- of the faces in sdq[face task][j].
template <int DIM, int P>
__device__ __forceinline__ void lifted_grad(const double* sq, const double* sdq, int l, int n, const int (&ii)[3],
                                            const double* sD, const double* sw, const Geo& g,
                                            double (&G)[DIM][DIM + 1]) {
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, NF = L::NF, EPB = L::EPB, NQ = DIM + 1, NFC = 2 * DIM;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int st = L::stride(d);
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const double* row = &sq[(j * EPB + l) * NP + n - ii[d] * st];
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < N1; ++k) s += sD[ii[d] * N1 + k] * row[k * st];
      G[d][j] = g.rh2[d] * s;
    }
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (ii[d] != (side ? P : 0)) continue;
      const double lift = g.rh2[d] / sw[ii[d]] * 0.5 * (side ? 1.0 : -1.0);
      const double* dq = &sdq[((l * NFC + 2 * d + side) * NF + face_index<DIM, N1>(d, ii)) * NQ];
#pragma unroll
      for (int j = 0; j < NQ; ++j) G[d][j] += lift * dq[j];
    }
}

// Face task k of a workgroup of EPB elements from e0: element slot l, face
// f = 2 d + side, face node fn; the node on the face (nown), the matching
// node of the neighbour (nn) and the neighbour (nb).
template <int DIM, int P>
struct FaceTask {
  using L = EL<DIM, P>;
  static constexpr int NF = L::NF, NFC = 2 * DIM;
  int l, f, fn, nown, nn, nb;
  __device__ FaceTask(int k, int e0, const Geo& g) {
    l = k / (NFC * NF);
    f = (k / NF) % NFC;
    fn = k % NF;
    const int d = f >> 1, side = f & 1;
    nown = face_node<DIM, L::N1>(d, fn, side ? P : 0);
    nn = face_node<DIM, L::N1>(d, fn, side ? 0 : P);
    nb = e0 + l < g.E ? neighbour(g, e0 + l, d, side ? 1 : -1) : 0;
  }
};

// The jumps q^+ - q^- at the face nodes of the workgroup's elements into
// sdq (uo0: the outside state of task threadIdx.x, loaded by the caller).
template <int DIM, int P>
__device__ __forceinline__ void face_jumps(const double* __restrict__ u, long vs, const EqP& q, const Geo& g, int e0,
                                           const double* sq, const double (&uo0)[DIM + 2], double* sdq) {
  using L = EL<DIM, P>;
  constexpr int NP = L::NP, NF = L::NF, EPB = L::EPB, NV = DIM + 2, NQ = DIM + 1, NTASK = EPB * 2 * DIM * NF;
  const int t = threadIdx.x;
  for (int k = t; k < NTASK; k += L::NTF) {
    const FaceTask<DIM, P> ft(k, e0, g);
    if (e0 + ft.l >= g.E) continue;
    double uo[NV], qn[NQ];
    for (int v = 0; v < NV; ++v) uo[v] = k == t ? uo0[v] : u[v * vs + (long)ft.nb * NP + ft.nn];
    prim_q<DIM>(q, uo, qn);
    for (int j = 0; j < NQ; ++j) sdq[k * NQ + j] = qn[j] - sq[(j * EPB + ft.l) * NP + ft.nown];
  }
}

// Pass 1 of the viscous term: the viscous fluxes f_v,d at face nodes,
// trace[v][e][d][side][f].
template <int DIM, int P>
__global__ void __launch_bounds__((EL<DIM, P>::NTF))
k_visc_trace(const double* __restrict__ u, double* __restrict__ trace, Geo g, EqP q, const double* __restrict__ tab,
             long vs) {
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, NF = L::NF, EPB = L::EPB, NV = DIM + 2, NQ = DIM + 1, NFC = 2 * DIM;
  constexpr int NTASK = EPB * NFC * NF;
  static_assert(L::NT >= N1 * N1, "a thread per entry of the tables");
  __shared__ double sD[N1 * N1], sw[N1];
  __shared__ double sq[NQ * EPB * NP], su[NV * EPB * NP];
  __shared__ double sdq[NTASK * NQ];
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB, e = e0 + le;
  const bool act = (le < EPB) && (e < g.E);
  double uu[NV], uo0[NV];
  for (int v = 0; v < NV; ++v) uu[v] = act ? u[v * vs + (long)e * NP + n] : 1.0;
  const double dv = t < N1 * N1 ? tab[t] : 0.0, wv = t < N1 ? tab[N1 * N1 + t] : 0.0;
  if (t < NTASK) {
    const FaceTask<DIM, P> ft(t, e0, g);
    for (int v = 0; v < NV; ++v) uo0[v] = e0 + ft.l < g.E ? u[v * vs + (long)ft.nb * NP + ft.nn] : 1.0;
  }
  if (t < N1 * N1) sD[t] = dv;
  if (t < N1) sw[t] = wv;
  if (act) {
    double qo[NQ];
    prim_q<DIM>(q, uu, qo);
    for (int j = 0; j < NQ; ++j) sq[(j * EPB + le) * NP + n] = qo[j];
    for (int v = 0; v < NV; ++v) su[(v * EPB + le) * NP + n] = uu[v];
  }
  __syncthreads();
  face_jumps<DIM, P>(u, vs, q, g, e0, sq, uo0, sdq);
  __syncthreads();
  // a face task per face node: the lifted gradient there and the flux
  // normal to its face
  for (int k = t; k < NTASK; k += L::NTF) {
    const FaceTask<DIM, P> ft(k, e0, g);
    if (e0 + ft.l >= g.E) continue;
    int jj[3];
    decomp<DIM, N1>(ft.nown, jj);
    double G[DIM][NQ], uf[NV];
    lifted_grad<DIM, P>(sq, sdq, ft.l, ft.nown, jj, sD, sw, g, G);
    for (int v = 0; v < NV; ++v) uf[v] = su[(v * EPB + ft.l) * NP + ft.nown];
    const int d = ft.f >> 1;
    double f[NV];
    if (d == 0)  // the axis as a constant, so that G stays in registers
      visc_flux<DIM>(q, 0, uf, G, f);
    else if (d == 1)
      visc_flux<DIM>(q, 1, uf, G, f);
    else
      visc_flux<DIM>(q, DIM - 1, uf, G, f);
    for (int v = 0; v < NV; ++v)
      trace[(((long)v * g.E + e0 + ft.l) * DIM + d) * 2 * NF + (ft.f & 1) * NF + ft.fn] = f[v];
  }
}

// Pass 2: out += V(u) = J w sum_d (2/h_d) D_d f_v,d + sum_faces J_f w_f
// ({f_v} - f_v^-).n  (accumulated onto out, which holds C(u)); with add
// != NULL, out = add + V(u) instead (add holds C(u), out is not read).
template <int DIM, int P>
__global__ void __launch_bounds__((EL<DIM, P>::NTF))
k_visc_apply(const double* __restrict__ u, double* __restrict__ out, const double* __restrict__ trace, Geo g, EqP q,
             const double* __restrict__ tab, long vs, const double* __restrict__ add) {
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, NF = L::NF, EPB = L::EPB, NV = DIM + 2, NQ = DIM + 1, NFC = 2 * DIM;
  constexpr int NTASK = EPB * NFC * NF;
  static_assert(L::NT >= N1 * N1, "a thread per entry of the tables");
  __shared__ double sD[N1 * N1], sw[N1];
  __shared__ double sq[NQ * EPB * NP];
  __shared__ double sf[NV * EPB * NP];
  __shared__ double sdq[NTASK * NQ];
  __shared__ double sfc[NTASK * NV];  // face corrections (component 0 unused)
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  const int e0 = xcd_block(blockIdx.x, gridDim.x) * EPB, e = e0 + le;
  const bool act = (le < EPB) && (e < g.E);
  // the node's state, the tables, and for face task t the neighbour's state
  // and its viscous flux on the shared face
  double uu[NV], uo0[NV], tr0[NV];
  for (int v = 0; v < NV; ++v) uu[v] = act ? u[v * vs + (long)e * NP + n] : 1.0;
  const double dv = t < N1 * N1 ? tab[t] : 0.0, wv = t < N1 ? tab[N1 * N1 + t] : 0.0;
  if (t < NTASK) {
    const FaceTask<DIM, P> ft(t, e0, g);
    const bool in = e0 + ft.l < g.E;
    const int d = ft.f >> 1, side = ft.f & 1;
    for (int v = 0; v < NV; ++v) {
      uo0[v] = in ? u[v * vs + (long)ft.nb * NP + ft.nn] : 1.0;
      tr0[v] = in && v > 0 ? trace[(((long)v * g.E + ft.nb) * DIM + d) * 2 * NF + (side ? 0 : NF) + ft.fn] : 0.0;
    }
  }
  if (t < N1 * N1) sD[t] = dv;
  if (t < N1) sw[t] = wv;
  int ii[3];
  decomp<DIM, N1>(n, ii);
  if (act) {
    double qo[NQ];
    prim_q<DIM>(q, uu, qo);
    for (int j = 0; j < NQ; ++j) sq[(j * EPB + le) * NP + n] = qo[j];
  }
  __syncthreads();
  face_jumps<DIM, P>(u, vs, q, g, e0, sq, uo0, sdq);
  __syncthreads();
  double G[DIM][NQ];
  if (act) lifted_grad<DIM, P>(sq, sdq, le, n, ii, sD, sw, g, G);
  double acc[NV];
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int d = 0; d < DIM; ++d) {
    if (act) {
      double f[NV];
      visc_flux<DIM>(q, d, uu, G, f);
      for (int v = 0; v < NV; ++v) sf[(v * EPB + le) * NP + n] = f[v];
    }
    __syncthreads();
    if (act) {
      const int st = L::stride(d);
      for (int v = 1; v < NV; ++v) {
        const double* row = &sf[(v * EPB + le) * NP + n - ii[d] * st];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < N1; ++k) s += sD[ii[d] * N1 + k] * row[k * st];
        acc[v] += g.rh2[d] * s;
      }
    }
    // the face corrections on the faces normal to d: J_f w_f (f^+ - f^-)/2 . n
    for (int k = t; k < NTASK; k += L::NTF) {
      const FaceTask<DIM, P> ft(k, e0, g);
      if (e0 + ft.l >= g.E || (ft.f >> 1) != d) continue;
      const int side = ft.f & 1;
      const double wf = DIM == 2 ? sw[ft.fn] : sw[ft.fn % N1] * sw[ft.fn / N1];
      const double jfwf = g.J * g.rh2[d] * wf;
      for (int v = 1; v < NV; ++v) {
        const double fnb =
            k == t ? tr0[v] : trace[(((long)v * g.E + ft.nb) * DIM + d) * 2 * NF + (side ? 0 : NF) + ft.fn];
        sfc[k * NV + v] = jfwf * 0.5 * (side ? 1.0 : -1.0) * (fnb - sf[(v * EPB + ft.l) * NP + ft.nown]);
      }
    }
    __syncthreads();
  }
  if (!act) return;
  double wn = 1.0;
  for (int d = 0; d < DIM; ++d) wn *= sw[ii[d]];
  for (int v = 0; v < NV; ++v) acc[v] *= g.J * wn;
  for (int d = 0; d < DIM; ++d)
    for (int side = 0; side < 2; ++side) {
      if (ii[d] != (side ? P : 0)) continue;
      const double* c = &sfc[((le * NFC + 2 * d + side) * NF + face_index<DIM, N1>(d, ii)) * NV];
      for (int v = 1; v < NV; ++v) acc[v] += c[v];
    }
  const long i0 = (long)e * NP + n;
  if (add) {
    out[i0] = add[i0];  // the mass row has no viscous term
    for (int v = 1; v < NV; ++v) out[v * vs + i0] = add[v * vs + i0] + acc[v];
  } else {
    for (int v = 1; v < NV; ++v) out[v * vs + i0] += acc[v];
  }
}

// ---------------------------------------------------------------- SIPG
template <typename T>
__device__ __forceinline__ T coef_w2(const CoefT<T>& cf, long idx) {
  if (cf.ub == nullptr) return cf.c;
  const T w = cf.ub[idx];
  return cf.c * w * w;
}

// nu + eps_e of element e (the isotropic part of D there)
template <typename T>
__device__ __forceinline__ T coef_nu(const CoefT<T>& cf, int e) {
  return cf.eps != nullptr ? cf.nu + cf.eps[e] : cf.nu;
}

// (D grad x)_d at the face nodes of one element from its LDS tile sx,
// stored in trace[c][e][d][side][f].
template <typename T, int DIM, int P>
__device__ __forceinline__ void store_trace(const T* sx, const T* sD, int n, const int (&ii)[3],
                                            T cw, const CoefT<T>& cf, const Geo& g, T* trace, int c,
                                            int e) {
  using L = EL<DIM, P>;
  const T rh2[3] = {(T)g.rh2[0], (T)g.rh2[1], (T)g.rh2[2]};
  constexpr int N1 = L::N1, NF = L::NF;
  bool face = false;
  for (int d = 0; d < DIM; ++d) face = face || ii[d] == 0 || ii[d] == P;
  if (!face) return;
  T gr[DIM];
  for (int d = 0; d < DIM; ++d) {
    const int st = L::stride(d);
    const T* row = &sx[n - ii[d] * st];
    T s = T(0.0);
#pragma unroll
    for (int k = 0; k < N1; ++k) s += sD[ii[d] * N1 + k] * row[k * st];
    gr[d] = rh2[d] * s;
  }
  T vg = T(0.0);
  for (int j = 0; j < DIM; ++j) vg += cf.v[j] * gr[j];
  for (int d = 0; d < DIM; ++d) {
    const bool lo = ii[d] == 0, hi = ii[d] == P;
    if (!lo && !hi) continue;
    const T qd = cw * cf.v[d] * vg + coef_nu(cf, e) * gr[d];
    const long base = (((long)c * g.E + e) * DIM + d) * 2 * NF + face_index<DIM, N1>(d, ii);
    if (lo) trace[base] = qd;
    if (hi) trace[base + NF] = qd;
  }
}

// Pass 1 of K_D x: the face traces of (D grad x).
template <typename T, int DIM, int P>
__global__ void __launch_bounds__((EL<DIM, P>::NT))
k_sipg_trace(const T* __restrict__ x, int nv, long vs, CoefT<T> cf, T* __restrict__ trace, Geo g,
             const T* __restrict__ tab) {
  const T rh2[3] = {(T)g.rh2[0], (T)g.rh2[1], (T)g.rh2[2]};
  const T gJ = (T)g.J;
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, EPB = L::EPB;
  __shared__ T sD[N1 * N1];
  __shared__ T sx[EPB * NP];
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  const int e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool act = (le < EPB) && (e < g.E);
  for (int k = t; k < N1 * N1; k += blockDim.x) sD[k] = tab[k];
  int ii[3];
  decomp<DIM, N1>(n, ii);
  const T cw = act ? coef_w2(cf, (long)e * NP + n) : T(0.0);
  for (int c = 0; c < nv; ++c) {
    __syncthreads();
    if (act) sx[le * NP + n] = x[c * vs + (long)e * NP + n];
    __syncthreads();
    if (act) store_trace<T, DIM, P>(&sx[le * NP], sD, n, ii, cw, cf, g, trace, c, e);
  }
}

// Pass 2: out = alpha M x + beta K_D x (weak SIPG).  With part != NULL the
// block partial of (out, dotv) is stored in part[blockIdx.x].  Blocks loop
// over tiles.  done_gen (nullable): skip when *done_gen == id.
template <typename T, int DIM, int P>
__global__ void __launch_bounds__((EL<DIM, P>::NT))
k_sipg_apply(const T* __restrict__ x, T* __restrict__ out, int nv, long vs, CoefT<T> cf,
             const T* __restrict__ trace, T alpha, T beta, T ctau, Geo g,
             const T* __restrict__ tab, const T* __restrict__ dotv, T* part,
             const int* __restrict__ done_gen, int id) {
  const T rh2[3] = {(T)g.rh2[0], (T)g.rh2[1], (T)g.rh2[2]};
  const T gJ = (T)g.J;
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, NF = L::NF, EPB = L::EPB;
  if (done_gen != nullptr && *done_gen == id) return;
  __shared__ T sD[N1 * N1], sw[N1];
  __shared__ T sx[EPB * NP];
  __shared__ T sQ[EPB * DIM * NP];
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  for (int k = t; k < N1 * N1; k += blockDim.x) sD[k] = tab[k];
  for (int k = t; k < N1; k += blockDim.x) sw[k] = tab[N1 * N1 + k];
  int ii[3];
  decomp<DIM, N1>(n, ii);
  __syncthreads();
  T wn = T(1.0);
  for (int d = 0; d < DIM; ++d) wn *= sw[ii[d]];
  const T jw = gJ * wn;
  const T pen = ctau * (T)(N1 * N1);
  const int ntiles = (g.E + EPB - 1) / EPB;
  T dacc = T(0.0);
  int tile0, tile1;
  tile_range(ntiles, tile0, tile1);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int e = tile * EPB + le;
    const bool act = (le < EPB) && (e < g.E);
    const long own = (long)e * NP + n;
    const T cw = act ? coef_w2(cf, own) : T(0.0);
    const T nue = act ? coef_nu(cf, e) : T(0.0);
    for (int c = 0; c < nv; ++c) {
      __syncthreads();
      if (act) sx[le * NP + n] = x[c * vs + own];
      __syncthreads();
      T r = T(0.0), xo = T(0.0);
      if (act) {
        xo = sx[le * NP + n];
        T gr[DIM];
        for (int d = 0; d < DIM; ++d) {
          const int st = L::stride(d);
          const T* row = &sx[le * NP + n - ii[d] * st];
          T s = T(0.0);
#pragma unroll
          for (int k = 0; k < N1; ++k) s += sD[ii[d] * N1 + k] * row[k * st];
          gr[d] = rh2[d] * s;
        }
        T vg = T(0.0);
        for (int j = 0; j < DIM; ++j) vg += cf.v[j] * gr[j];
        T qv[DIM], Qd[DIM];
        for (int d = 0; d < DIM; ++d) {
          qv[d] = cw * cf.v[d] * vg + nue * gr[d];
          Qd[d] = jw * qv[d];
        }
        for (int d = 0; d < DIM; ++d) {
          for (int side = 0; side < 2; ++side) {
            if (ii[d] != (side ? P : 0)) continue;
            const T sgn = side ? T(1.0) : -T(1.0);
            const int nb = neighbour(g, e, d, side ? 1 : -1);
            const int nn = n + ((side ? 0 : P) - ii[d]) * L::stride(d);
            const long nbi = (long)nb * NP + nn;
            const T xnb = x[c * vs + nbi];
            const T qnb = trace[(((long)c * g.E + nb) * DIM + d) * 2 * NF + (side ? 0 : NF) +
                                     face_index<DIM, N1>(d, ii)];
            const T dnb = coef_w2(cf, nbi) * cf.v[d] * cf.v[d] + coef_nu(cf, nb);
            const T dow = cw * cf.v[d] * cf.v[d] + nue;
            const T qn = T(0.5) * sgn * (qv[d] + qnb);
            const T tau = pen * fmax(dow, dnb) * T(0.5) * rh2[d];
            const T jump = xo - xnb;
            const T jfwf = gJ * rh2[d] * wn / sw[ii[d]];
            r += jfwf * (-qn + tau * jump);
            for (int d2 = 0; d2 < DIM; ++d2)
              Qd[d2] -= T(0.5) * jfwf * jump * sgn * (cw * cf.v[d2] * cf.v[d] + (d2 == d ? nue : T(0.0)));
          }
        }
        for (int d = 0; d < DIM; ++d) sQ[(le * DIM + d) * NP + n] = Qd[d];
      }
      __syncthreads();
      if (act) {
        for (int d = 0; d < DIM; ++d) {
          const int st = L::stride(d);
          const T* row = &sQ[(le * DIM + d) * NP + n - ii[d] * st];
          T s = T(0.0);
#pragma unroll
          for (int k = 0; k < N1; ++k) s += sD[k * N1 + ii[d]] * row[k * st];
          r += rh2[d] * s;
        }
        const T val = alpha * jw * xo + beta * r;
        out[c * vs + own] = val;
        if (dotv != nullptr) dacc += val * dotv[c * vs + own];
      }
    }
  }
  if (part != nullptr) {
    const T v1[1] = {dacc};
    T* const pp[1] = {part};
    block_partials<T, 1>(v1, pp);
  }
}

// ---------------------------------------------------------------- SIPG, isotropic, hexahedra
// K_D x for an isotropic coefficient D = nu I that is constant on the level
// (the systems' kappa_m I; a scalar problem without convection) on
// hexahedra with (P+1)^2 dividing 64.  With D isotropic the flux along axis
// d involves only the derivative along d, so the operator splits into three
// one-dimensional problems: for each axis, gradient, flux, the face terms
// of the two faces normal to that axis and the transposed contraction act
// on the P+1 nodes of a grid line.  The neighbour's face flux is the
// derivative of the neighbour's own line, so no face-trace pass is needed.
//
// A group of (P+1)^2 lanes owns one (component, element) pair; for every
// axis in turn lane l of the group holds, in registers, the line through
// (a, b) = (l mod (P+1), l div (P+1)) along that axis, and the lines of the
// two neighbours across the faces it ends on (loaded from global memory:
// all three line layouts are coalesced).  The contributions of the three
// axes are summed in an LDS region of the group (rows padded to P+2 to
// spread the banks).  A group lies inside one wave, so the LDS exchange
// needs no workgroup barrier; waves work on their own pairs.
//
// The operand is x, or x scaled node by node by isc[n] (isc holds NP values,
// the same for every element and component: the inverse Jacobi diagonal of
// an isotropic operator).  out = alpha M x + beta K_D x; with part != NULL
// the block partial of (out, operand) is stored in part[blockIdx.x];
// done_gen (nullable): skip when *done_gen == id.
template <int P>
struct ISO {
  static constexpr int N1 = P + 1, NP = N1 * N1 * N1, LG = N1 * N1, GW = 64 / LG;
  static constexpr int WAVES = P >= 7 ? 16 : 4;       // waves per workgroup
  static constexpr int NT = 64 * WAVES, GPB = GW * WAVES;  // threads, groups per workgroup
  static constexpr int SY = N1 + 1, SZ = N1 * SY, REG = N1 * SZ;  // padded LDS region of a group
  static_assert(64 % LG == 0, "the lane groups must tile a wave");
};

// node index of position k on the grid line along axis D through (a, b)
template <int D, int N1>
__device__ __forceinline__ int line_node(int k, int a, int b) {
  return D == 0 ? k + N1 * (a + N1 * b) : (D == 1 ? a + N1 * (k + N1 * b) : a + N1 * (b + N1 * k));
}

// Orders the LDS accesses of a wave: stores issued before are seen by the
// loads of every lane of the wave issued after.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The operand on the line (a, b) along D of element e (component base xc),
// scaled by the LDS table sc when `scaled`.
// A line along axis 0 is contiguous and 16-byte aligned when 16 / sizeof(T)
// divides P+1 (vectors start 256-byte aligned, an element holds (P+1)^3
// values): it is then read with 16-byte loads, which touch a quarter (FP64)
// of the cache lines per instruction that 8-byte loads at a lane stride of
// P+1 values would.
template <typename T, int P, int D>
__device__ __forceinline__ void load_line(const T* __restrict__ xc, int e, int a, int b, const T* sc, bool scaled,
                                          T (&v)[P + 1]) {
  constexpr int N1 = P + 1, NP = N1 * N1 * N1;
  constexpr int VW = 16 / (int)sizeof(T);  // values per 16-byte load
  const T* const xe = xc + (long)e * NP;
  if constexpr (D == 0 && N1 % VW == 0) {
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    const V* const lv = reinterpret_cast<const V*>(xe + line_node<0, N1>(0, a, b));
#pragma unroll
    for (int q = 0; q < N1 / VW; ++q) {
      const V t = lv[q];
      const T* const tt = reinterpret_cast<const T*>(&t);
#pragma unroll
      for (int i = 0; i < VW; ++i) v[q * VW + i] = tt[i];
    }
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) v[k] = xe[line_node<D, N1>(k, a, b)];
  }
  if (scaled) {
#pragma unroll
    for (int k = 0; k < N1; ++k) v[k] *= sc[line_node<D, N1>(k, a, b)];
  }
}

// Axis D of the isotropic apply on the line (a, b) of element e: xl holds
// the operand on the line; r[k] receives the volume and face terms of line
// node k.

// D[k][j] and w[k] of degree P as literal constants of type T
template <typename T, int P, int K, int J>
__device__ __forceinline__ constexpr T gll_d() {
  constexpr T v = (T)kGLL<P>.D[K][J];
  return v;
}
template <typename T, int P, int K>
__device__ __forceinline__ constexpr T gll_w() {
  constexpr T v = (T)kGLL<P>.w[K];
  return v;
}

// Axis D of the isotropic apply on one grid line, the neighbours' lines
// across the two faces given (nlm: minus side, nlp: plus side).
template <typename T, int P, int D>
__device__ __forceinline__ void iso_axis_nl(const T (&xl)[P + 1], const T (&nlm)[P + 1], const T (&nlp)[P + 1],
                                            T (&r)[P + 1], const Geo& g, T nu, T pen, T wab) {
  constexpr int N1 = P + 1;
  const T rh = (T)g.rh2[D], J = (T)g.J;
  T q[N1], Q[N1];
  static_for<N1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    T s = T(0.0);
    static_for<N1>([&](auto jc) { s += gll_d<T, P, k, decltype(jc)::value>() * xl[decltype(jc)::value]; });
    q[k] = nu * rh * s;  // flux along D
    Q[k] = J * wab * gll_w<T, P, k>() * q[k];
  });
  const T jfwf = J * rh * wab;
  const T tau = pen * nu * T(0.5) * rh;
  static_for<2>([&](auto sidec) {
    constexpr int side = decltype(sidec)::value;
    constexpr int ke = side ? P : 0;   // this element's node on the face
    constexpr int kn = side ? 0 : P;   // the neighbour's node on the face
    const T sgn = side ? T(1.0) : -T(1.0);
    const T(&nl)[N1] = side ? nlp : nlm;
    T sn = T(0.0);
    static_for<N1>([&](auto jc) { sn += gll_d<T, P, kn, decltype(jc)::value>() * nl[decltype(jc)::value]; });
    const T qn = T(0.5) * sgn * (q[ke] + nu * rh * sn);
    const T jump = xl[ke] - nl[kn];
    r[ke] += jfwf * (-qn + tau * jump);
    Q[ke] -= T(0.5) * jfwf * jump * sgn * nu;
  });
  static_for<N1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    T s = T(0.0);
    static_for<N1>([&](auto jc) { s += gll_d<T, P, decltype(jc)::value, k>() * Q[decltype(jc)::value]; });
    r[k] += rh * s;
  });
}

// Axis D with the neighbours' lines loaded from global memory.
template <typename T, int P, int D>
__device__ __forceinline__ void iso_axis(const T* __restrict__ xc, const T* sc, bool scaled,
                                         const T (&xl)[P + 1], T (&r)[P + 1], int nbm, int nbp, int a, int b,
                                         const Geo& g, T nu, T pen, T wab) {
  T nlm[P + 1], nlp[P + 1];
  load_line<T, P, D>(xc, nbm, a, b, sc, scaled, nlm);
  load_line<T, P, D>(xc, nbp, a, b, sc, scaled, nlp);
  iso_axis_nl<T, P, D>(xl, nlm, nlp, r, g, nu, pen, wab);
}

template <typename T, int P>
__global__ void __launch_bounds__((ISO<P>::NT))
k_sipg_apply_iso3(const T* __restrict__ x, const T* __restrict__ isc, T* __restrict__ out, int nv, long vs, T nu,
                  T alpha, T beta, T ctau, Geo g, const T* __restrict__ tab, T* part,
                  const int* __restrict__ done_gen, int id) {
  using I = ISO<P>;
  constexpr int N1 = I::N1, LG = I::LG, SY = I::SY, SZ = I::SZ, REG = I::REG;
  if (done_gen != nullptr && *done_gen == id) return;
  __shared__ T sR[I::GPB * REG];
  // one group per wave (P = 7): the pair, its element and its neighbours are
  // wave-uniform and live in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = I::GW == 1 ? 0 : lane / LG, l = lane - grp * LG;
  const int a = l % N1, b = l / N1;
  T* const R = &sR[(wave * I::GW + grp) * REG];
  const T* const w = tab + N1 * N1;  // GLL weights (runtime table: lane-dependent index)
  const T pen = ctau * (T)(N1 * N1), J = (T)g.J;
  const T wab[3] = {w[b] * w[a], w[a] * w[b], w[a] * w[b]};  // line weights w_a w_b per axis
  __shared__ T sc[I::NP];  // operand scale per node
  const bool scaled = isc != nullptr;
  if (scaled)
    for (int k = threadIdx.x; k < I::NP; k += blockDim.x) sc[k] = isc[k];
  __syncthreads();
  // Every XCD takes one contiguous range of pairs (a slab of elements); its
  // workgroups interleave over that range group by group, so the pairs in
  // flight on an XCD at any time are a compact window and the neighbour
  // lines they read were loaded into that XCD's L2 by the same window.
  const long npairs = (long)nv * g.E;
  const int G = gridDim.x, xcd = blockIdx.x % kXcd, per = G / kXcd, rem = G % kXcd;
  const long kx = per + (xcd < rem ? 1 : 0);                  // workgroups of this XCD
  const long lb0 = (long)xcd * per + (xcd < rem ? xcd : rem); // its first logical id
  const long xs = lb0 * npairs / G, xe = (lb0 + kx) * npairs / G;
  const long k = blockIdx.x / kXcd;                           // rank among them
  T dacc = T(0.0);
  for (long p = xs + k * I::GPB + wave * I::GW + grp; p < xe; p += kx * I::GPB) {
    const int c = (int)(p / g.E), e = (int)(p - (long)c * g.E);
    const int ex = e % g.ne[0], ey = (e / g.ne[0]) % g.ne[1], ez = e / (g.ne[0] * g.ne[1]);
    const int sx = 1, sy = g.ne[0], sz = g.ne[0] * g.ne[1];
    // neighbours across the faces normal to each axis (periodic)
    const int nbm0 = e + (ex > 0 ? -sx : (g.ne[0] - 1) * sx), nbp0 = e + (ex < g.ne[0] - 1 ? sx : -(g.ne[0] - 1) * sx);
    const int nbm1 = e + (ey > 0 ? -sy : (g.ne[1] - 1) * sy), nbp1 = e + (ey < g.ne[1] - 1 ? sy : -(g.ne[1] - 1) * sy);
    const int ezl = ez % g.wl;  // position inside the instance along z
    const int nbm2 = e + (ezl > 0 ? -sz : (g.wl - 1) * sz), nbp2 = e + (ezl < g.wl - 1 ? sz : -(g.wl - 1) * sz);
    const T* const xc = x + c * vs;
    T xl[N1], r[N1];
    load_line<T, P, 0>(xc, e, a, b, sc, scaled, xl);
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = T(0.0);
    iso_axis<T, P, 0>(xc, sc, scaled, xl, r, nbm0, nbp0, a, b, g, nu, pen, wab[0]);
#pragma unroll
    for (int k = 0; k < N1; ++k) R[k + SY * a + SZ * b] = r[k];
    wave_lds_fence();
    load_line<T, P, 1>(xc, e, a, b, sc, scaled, xl);
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = T(0.0);
    iso_axis<T, P, 1>(xc, sc, scaled, xl, r, nbm1, nbp1, a, b, g, nu, pen, wab[1]);
#pragma unroll
    for (int k = 0; k < N1; ++k) R[a + SY * k + SZ * b] += r[k];
    wave_lds_fence();
    load_line<T, P, 2>(xc, e, a, b, sc, scaled, xl);
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = T(0.0);
    iso_axis<T, P, 2>(xc, sc, scaled, xl, r, nbm2, nbp2, a, b, g, nu, pen, wab[2]);
    const T jab = J * w[a] * w[b];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const T val = alpha * jab * w[k] * xl[k] + beta * (r[k] + R[a + SY * b + SZ * k]);
      out[c * vs + (long)e * I::NP + line_node<2, N1>(k, a, b)] = val;
      dacc += val * xl[k];
    }
    wave_lds_fence();  // the next pair's stores follow these loads
  }
  if (part != nullptr) {
    const T v1[1] = {dacc};
    T* const pp[1] = {part};
    block_partials<T, 1>(v1, pp);
  }
}

// The isotropic apply on hexahedra with P = 7 (one wave per element, a lane
// per grid line) for meshes with an even number of elements along every
// axis, by 2 x 2 x 2 bricks: a workgroup of 8 waves takes one brick of one
// component at a time, loads the brick's 8 elements once into LDS (padded
// rows, so that lines along any axis are read with at most 3-way bank
// conflicts), and reads every line of an element and of the neighbour inside
// the brick from there; only the neighbour outside the brick, one per axis,
// comes from global memory (the first axis's lines are requested before the
// brick is staged).  Per element that is 4 element-sized reads through the
// cache hierarchy instead of 9 (own element once per axis, both neighbours
// per axis).  Same operator, operand scaling, output and partials as
// k_sipg_apply_iso3; bricks are numbered x fastest and every XCD takes a
// contiguous range of (component, brick) tasks.
template <int P>
struct ISOB {
  static constexpr int N1 = P + 1, NP = N1 * N1 * N1;
  static constexpr int SY = N1 + 1, SZ = N1 * SY, REG = N1 * SZ;  // padded element layout in LDS
  static constexpr int NT = 8 * 64;
  static_assert(N1 * N1 == 64, "one lane per grid line of a wave");
};

template <typename T, int P, int D>
__device__ __forceinline__ void lds_line(const T* el, int a, int b, T (&v)[P + 1]) {
  using I = ISOB<P>;
#pragma unroll
  for (int k = 0; k < P + 1; ++k)
    v[k] = el[D == 0 ? k + I::SY * a + I::SZ * b : (D == 1 ? a + I::SY * k + I::SZ * b : a + I::SY * b + I::SZ * k)];
}

template <typename T, int P>
__global__ void __launch_bounds__((ISOB<P>::NT), 4)
k_sipg_apply_iso3_brick(const T* __restrict__ x, const T* __restrict__ isc, T* __restrict__ out, int nv, long vs,
                        T nu, T alpha, T beta, T ctau, Geo g, const T* __restrict__ tab, T* part,
                        const int* __restrict__ done_gen, int id) {
  using I = ISOB<P>;
  constexpr int N1 = I::N1, NP = I::NP, SY = I::SY, SZ = I::SZ, REG = I::REG;
  if (done_gen != nullptr && *done_gen == id) return;
  __shared__ T sX[8 * REG];  // the brick's operand, element w at sX + w REG
  __shared__ T sR[8 * REG];  // per wave: the axis contributions of its element
  __shared__ T sc[NP];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int a = lane % N1, b = lane / N1;
  const int bx = wave & 1, by = (wave >> 1) & 1, bz = wave >> 2;
  T* const R = &sR[wave * REG];
  T* const X = &sX[wave * REG];
  const T* const w = tab + N1 * N1;
  const T pen = ctau * (T)(N1 * N1), J = (T)g.J;
  const T wab[3] = {w[b] * w[a], w[a] * w[b], w[a] * w[b]};
  const bool scaled = isc != nullptr;
  for (int k = threadIdx.x; k < NP; k += blockDim.x) sc[k] = scaled ? isc[k] : T(1.0);
  __syncthreads();
  const int nbx = g.ne[0] / 2, nby = g.ne[1] / 2, nbz = g.ne[2] / 2;
  const long nbr = (long)nbx * nby * nbz, ntask = (long)nv * nbr;
  const int G = gridDim.x, xcd = blockIdx.x % kXcd, per = G / kXcd, rem = G % kXcd;
  const long kx = per + (xcd < rem ? 1 : 0);
  const long lb0 = (long)xcd * per + (xcd < rem ? xcd : rem);
  const long ts = lb0 * ntask / G, te = (lb0 + kx) * ntask / G;
  // The task index t = ((c nbz + Bz) nby + By) nbx + Bx is decoded once; the
  // stride kx is added digit by digit with carries, which keeps divisions out
  // of the loop (each digit of kx is below its radix, so one carry suffices).
  long t = ts + blockIdx.x / kXcd;
  int c = (int)(t / nbr), Bx, By, Bz;
  {
    const long br = t - (long)c * nbr;
    Bx = (int)(br % nbx), By = (int)((br / nbx) % nby), Bz = (int)(br / ((long)nbx * nby));
  }
  const int dc = (int)(kx / nbr), dx = (int)((kx % nbr) % nbx), dy = (int)(((kx % nbr) / nbx) % nby),
            dz = (int)((kx % nbr) / ((long)nbx * nby));
  T dacc = T(0.0);
  for (; t < te; t += kx) {
    const int ex = 2 * Bx + bx, ey = 2 * By + by, ez = 2 * Bz + bz;
    const int e = ex + g.ne[0] * (ey + g.ne[1] * ez);
    // the neighbour outside the brick along each axis (periodic)
    const int ox = bx ? (ex + 1 == g.ne[0] ? 0 : ex + 1) : (ex == 0 ? g.ne[0] - 1 : ex - 1);
    const int oy = by ? (ey + 1 == g.ne[1] ? 0 : ey + 1) : (ey == 0 ? g.ne[1] - 1 : ey - 1);
    const int ezl = ez % g.wl, ez0 = ez - ezl;  // bricks do not straddle instances (g.wl even)
    const int oz = ez0 + (bz ? (ezl + 1 == g.wl ? 0 : ezl + 1) : (ezl == 0 ? g.wl - 1 : ezl - 1));
    const int nx = ox + g.ne[0] * (ey + g.ne[1] * ez);
    const int ny = ex + g.ne[0] * (oy + g.ne[1] * ez);
    const int nz = ex + g.ne[0] * (ey + g.ne[1] * oz);
    const T* const xc = x + c * vs;
    T ext[N1];
    load_line<T, P, 0>(xc, nx, a, b, sc, scaled, ext);
    // stage the element (scaled) into the brick: lane holds node q 64 + lane
    {
      const T* const xe = xc + (long)e * NP;
#pragma unroll
      for (int q = 0; q < N1; ++q) {
        const int n = q * 64 + lane;
        X[(n % N1) + SY * ((n / N1) % N1) + SZ * q] = xe[n] * sc[n];
      }
    }
    __syncthreads();  // the brick is staged
    T xl[N1], nl[N1], r[N1];
    // axis 0: the neighbour inside the brick is wave ^ 1
    lds_line<T, P, 0>(X, a, b, xl);
    lds_line<T, P, 0>(&sX[(wave ^ 1) * REG], a, b, nl);
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = T(0.0);
    if (bx) iso_axis_nl<T, P, 0>(xl, nl, ext, r, g, nu, pen, wab[0]);
    else    iso_axis_nl<T, P, 0>(xl, ext, nl, r, g, nu, pen, wab[0]);
#pragma unroll
    for (int k = 0; k < N1; ++k) R[k + SY * a + SZ * b] = r[k];
    wave_lds_fence();
    // axis 1: wave ^ 2
    load_line<T, P, 1>(xc, ny, a, b, sc, scaled, ext);
    lds_line<T, P, 1>(X, a, b, xl);
    lds_line<T, P, 1>(&sX[(wave ^ 2) * REG], a, b, nl);
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = T(0.0);
    if (by) iso_axis_nl<T, P, 1>(xl, nl, ext, r, g, nu, pen, wab[1]);
    else    iso_axis_nl<T, P, 1>(xl, ext, nl, r, g, nu, pen, wab[1]);
#pragma unroll
    for (int k = 0; k < N1; ++k) R[a + SY * k + SZ * b] += r[k];
    wave_lds_fence();
    // axis 2: wave ^ 4, then the mass term and the output along z-lines
    load_line<T, P, 2>(xc, nz, a, b, sc, scaled, ext);
    lds_line<T, P, 2>(X, a, b, xl);
    lds_line<T, P, 2>(&sX[(wave ^ 4) * REG], a, b, nl);
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = T(0.0);
    if (bz) iso_axis_nl<T, P, 2>(xl, nl, ext, r, g, nu, pen, wab[2]);
    else    iso_axis_nl<T, P, 2>(xl, ext, nl, r, g, nu, pen, wab[2]);
    const T jab = J * w[a] * w[b];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const T val = alpha * jab * w[k] * xl[k] + beta * (r[k] + R[a + SY * b + SZ * k]);
      __builtin_nontemporal_store(val, &out[c * vs + (long)e * NP + line_node<2, N1>(k, a, b)]);
      dacc += val * xl[k];
    }
    __syncthreads();  // every wave is done with the brick and its R region
    Bx += dx;
    int cy = Bx >= nbx ? 1 : 0;
    Bx -= cy * nbx;
    By += dy + cy;
    cy = By >= nby ? 1 : 0;
    By -= cy * nby;
    Bz += dz + cy;
    cy = Bz >= nbz ? 1 : 0;
    Bz -= cy * nbz;
    c += dc + cy;
  }
  if (part != nullptr) {
    const T v1[1] = {dacc};
    T* const pp[1] = {part};
    block_partials<T, 1>(v1, pp);
  }
}

// The same isotropic apply on quadrilaterals: a group of P+1 lanes owns a
// (component, element) pair (64 / (P+1) groups per wave, the remaining lanes
// idle), lane a holding, for each of the two axes, the line through a.
template <int P>
struct ISO2 {
  static constexpr int N1 = P + 1, NP = N1 * N1, LG = N1, GW = 64 / N1;
  static constexpr int WAVES = 8;
  static constexpr int NT = 64 * WAVES, GPB = GW * WAVES;
  static constexpr int SY = N1 + 1, REG = N1 * SY;  // padded LDS region of a group
};

template <int D, int N1>
__device__ __forceinline__ int line_node2(int k, int a) {
  return D == 0 ? k + N1 * a : a + N1 * k;
}

template <typename T, int P, int D>
__device__ __forceinline__ void load_line2(const T* __restrict__ xc, int e, int a, const T* sc, bool scaled,
                                           T (&v)[P + 1]) {
  constexpr int N1 = P + 1, NP = N1 * N1;
  const T* const xe = xc + (long)e * NP;
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const int n = line_node2<D, N1>(k, a);
    v[k] = scaled ? xe[n] * sc[n] : xe[n];
  }
}

// Axis D on the line a of element e (neighbours nbm, nbp across the faces
// normal to D); wl = w_a, the weight of the line's other coordinate.
template <typename T, int P, int D>
__device__ __forceinline__ void iso_axis2(const T* __restrict__ xc, const T* sc, bool scaled, const T (&xl)[P + 1],
                                          T (&r)[P + 1], int nbm, int nbp, int a, const Geo& g, T nu, T pen, T wl) {
  constexpr int N1 = P + 1;
  const T rh = (T)g.rh2[D], J = (T)g.J;
  T q[N1], Q[N1];
  static_for<N1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    T s = T(0.0);
    static_for<N1>([&](auto jc) { s += gll_d<T, P, k, decltype(jc)::value>() * xl[decltype(jc)::value]; });
    q[k] = nu * rh * s;
    Q[k] = J * wl * gll_w<T, P, k>() * q[k];
  });
  const T jfwf = J * rh * wl;
  const T tau = pen * nu * T(0.5) * rh;
  static_for<2>([&](auto sidec) {
    constexpr int side = decltype(sidec)::value;
    constexpr int ke = side ? P : 0;
    constexpr int kn = side ? 0 : P;
    const T sgn = side ? T(1.0) : -T(1.0);
    T nl[N1];
    load_line2<T, P, D>(xc, side ? nbp : nbm, a, sc, scaled, nl);
    T sn = T(0.0);
    static_for<N1>([&](auto jc) { sn += gll_d<T, P, kn, decltype(jc)::value>() * nl[decltype(jc)::value]; });
    const T qn = T(0.5) * sgn * (q[ke] + nu * rh * sn);
    const T jump = xl[ke] - nl[kn];
    r[ke] += jfwf * (-qn + tau * jump);
    Q[ke] -= T(0.5) * jfwf * jump * sgn * nu;
  });
  static_for<N1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    T s = T(0.0);
    static_for<N1>([&](auto jc) { s += gll_d<T, P, decltype(jc)::value, k>() * Q[decltype(jc)::value]; });
    r[k] += rh * s;
  });
}

template <typename T, int P>
__global__ void __launch_bounds__((ISO2<P>::NT))
k_sipg_apply_iso2(const T* __restrict__ x, const T* __restrict__ isc, T* __restrict__ out, int nv, long vs, T nu,
                  T alpha, T beta, T ctau, Geo g, const T* __restrict__ tab, T* part,
                  const int* __restrict__ done_gen, int id, const T* __restrict__ addv) {
  using I = ISO2<P>;
  constexpr int N1 = I::N1, LG = I::LG, SY = I::SY, REG = I::REG;
  if (done_gen != nullptr && *done_gen == id) return;
  __shared__ T sR[I::GPB * REG];
  __shared__ T sc[I::NP];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = lane / LG, a = lane - grp * LG;
  const bool lane_on = grp < I::GW;
  T* const R = &sR[(wave * I::GW + (lane_on ? grp : 0)) * REG];
  const T* const w = tab + N1 * N1;
  const T pen = ctau * (T)(N1 * N1), J = (T)g.J;
  const T wa = w[lane_on ? a : 0];
  const bool scaled = isc != nullptr;
  if (scaled)
    for (int k = threadIdx.x; k < I::NP; k += blockDim.x) sc[k] = isc[k];
  __syncthreads();
  const long npairs = (long)nv * g.E;
  const int G = gridDim.x, xcd = blockIdx.x % kXcd, per = G / kXcd, rem = G % kXcd;
  const long kx = per + (xcd < rem ? 1 : 0);
  const long lb0 = (long)xcd * per + (xcd < rem ? xcd : rem);
  const long xs = lb0 * npairs / G, xe = (lb0 + kx) * npairs / G;
  const long kk = blockIdx.x / kXcd;
  T dacc = T(0.0);
  for (long p = xs + kk * I::GPB + wave * I::GW + grp; lane_on && p < xe; p += kx * I::GPB) {
    const int c = (int)(p / g.E), e = (int)(p - (long)c * g.E);
    const int ex = e % g.ne[0], ey = e / g.ne[0];
    const int sy = g.ne[0];
    const int nbm0 = e + (ex > 0 ? -1 : g.ne[0] - 1), nbp0 = e + (ex < g.ne[0] - 1 ? 1 : -(g.ne[0] - 1));
    const int eyl = ey % g.wl;  // position inside the instance along y
    const int nbm1 = e + (eyl > 0 ? -sy : (g.wl - 1) * sy), nbp1 = e + (eyl < g.wl - 1 ? sy : -(g.wl - 1) * sy);
    const T* const xc = x + c * vs;
    T xl[N1], r[N1];
    load_line2<T, P, 0>(xc, e, a, sc, scaled, xl);
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = T(0.0);
    iso_axis2<T, P, 0>(xc, sc, scaled, xl, r, nbm0, nbp0, a, g, nu, pen, wa);
#pragma unroll
    for (int k = 0; k < N1; ++k) R[k + SY * a] = r[k];
    wave_lds_fence();
    load_line2<T, P, 1>(xc, e, a, sc, scaled, xl);
#pragma unroll
    for (int k = 0; k < N1; ++k) r[k] = T(0.0);
    iso_axis2<T, P, 1>(xc, sc, scaled, xl, r, nbm1, nbp1, a, g, nu, pen, wa);
    const T ja = J * wa;
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const long oi = c * vs + (long)e * I::NP + line_node2<1, N1>(k, a);
      T val = alpha * ja * w[k] * xl[k] + beta * (r[k] + R[a + SY * k]);
      if (addv != nullptr) val = addv[oi] + val;
      out[oi] = val;
      dacc += val * xl[k];
    }
    wave_lds_fence();
  }
  if (part != nullptr) {
    const T v1[1] = {dacc};
    T* const pp[1] = {part};
    block_partials<T, 1>(v1, pp);
  }
}

template <typename T, int DIM, int P>
struct IsoKernel;  // the matvec kernel, its block size and lane groups per block
template <typename T, int P>
struct IsoKernel<T, 3, P> {
  static constexpr int NT = ISO<P>::NT, GPB = ISO<P>::GPB;
  static const void* fn() { return (const void*)k_sipg_apply_iso3<T, P>; }
};
template <typename T, int P>
struct IsoKernel<T, 2, P> {
  static constexpr int NT = ISO2<P>::NT, GPB = ISO2<P>::GPB;
  static const void* fn() { return (const void*)k_sipg_apply_iso2<T, P>; }
};

// NP-periodic inverse of the Jacobi diagonal of an isotropic operator (the
// diagonal is the same for every element and component): idg[n] = 1/diag[n].
template <typename T>
__global__ void k_inv_table(const T* __restrict__ diag, T* __restrict__ idg, int np) {
  for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < np; n += gridDim.x * blockDim.x) idg[n] = T(1.0) / diag[n];
}

// Per-thread sums by component over a flat vector in components of vs
// values, for a thread striding upwards through its range: the running sum
// of the current component is folded into acc[c] only when the index passes
// into the next component (at most a few times per thread).
template <typename T>
struct CompSum {
  T acc[kMaxComp];
  T cur;
  int c;
  long next;
  __device__ __forceinline__ void init(long vs) {
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) acc[k] = T(0.0);
    cur = T(0.0);
    c = 0;
    next = vs;
  }
  __device__ __forceinline__ void fold() {
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) acc[k] += k == c ? cur : T(0.0);
    cur = T(0.0);
  }
  __device__ __forceinline__ void add(long i, long vs, T v) {
    if (i >= next) {
      fold();
      while (i >= next) {
        ++c;
        next += vs;
      }
    }
    cur += v;
  }
};

// Jacobi-PCG (Chronopoulos-Gear) for the isotropic operator, streaming form:
// z = r idg is never stored (the matvec scales r itself), so an iteration
// moves r, w, p, s, x in and r, p, s, x out, with no face traces.  Same
// partial-sum protocol and stopping test as k_cg_start / k_cg_iter; blocks
// take contiguous ranges of the flattened vectors.
// With cg.b == NULL the right-hand side is the combination bl, formed node
// by node here (mw: the element's NP mass weights), so no assembly pass
// writes it first.
template <typename T, int NP>
__global__ void __launch_bounds__(1024)
k_cg_start_iso(CGStateT<T> cg, const T* __restrict__ idg, long n, LinComb bl, const double* __restrict__ mw) {
  T a[3] = {T(0.0), T(0.0), T(0.0)};
  CompSum<T> sb, sw;  // conservation: sum b and sum A x0 by component
  sb.init(cg.vs);
  sw.init(cg.vs);
  const long lb = xcd_block(blockIdx.x, gridDim.x);
  const long i0 = lb * n / gridDim.x, i1 = (lb + 1) * n / gridDim.x;
  if (cg.cons && threadIdx.x < kMaxComp) cg.cons[(10 + threadIdx.x) * cg.cap + blockIdx.x] = T(0.0);
  for (long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    T bi;
    if (cg.b) {
      bi = cg.b[i];
    } else {
      const double m = mw[i % NP];
      double v = 0.0;
      for (int j = 0; j < bl.n; ++j) v += bl.c[j] * (bl.m[j] ? m : 1.0) * bl.x[j][i];
      bi = (T)v;
    }
    const T wi = cg.w[i];
    const T ri = bi - wi;
    const T zi = ri * idg[i % NP];
    cg.r[i] = ri;
    a[0] += ri * zi;
    a[1] += ri * ri;
    a[2] += bi * bi;
    if (cg.cons) {
      sb.add(i, cg.vs, bi);
      sw.add(i, cg.vs, wi);
    }
  }
  T* const pp[3] = {cg.gam, cg.rr, cg.bbp};
  block_partials<T, 3>(a, pp);
  if (cg.cons) {  // uniform over the grid
    sb.fold();
    sw.fold();
    T* const pb[kMaxComp] = {cg.cons, cg.cons + cg.cap, cg.cons + 2 * cg.cap, cg.cons + 3 * cg.cap,
                             cg.cons + 4 * cg.cap};
    block_partials<T, kMaxComp>(sb.acc, pb);
    T* const pw[kMaxComp] = {cg.cons + 5 * cg.cap, cg.cons + 6 * cg.cap, cg.cons + 7 * cg.cap, cg.cons + 8 * cg.cap,
                             cg.cons + 9 * cg.cap};
    block_partials<T, kMaxComp>(sw.acc, pw);
  }
}

// ZS: z is stored (block-Jacobi preconditioner); CONS: conservation sums.
// Both are template flags, so the plain form's loop carries no test of them.
template <typename T, int NP, bool ZS, bool CONS>
__global__ void __launch_bounds__(1024)
k_cg_iter_iso(CGStateT<T> cg, const T* __restrict__ idg, long n, int it, int id, int nparts, int ndel) {
  if (*cg.done_gen == id) return;
  const int cap = cg.cap;
  T tot[4], dtot[1];
  {
    // this kernel's own partials (nparts), and the matvec's (w, z) partials (ndel)
    const T* const pr[4] = {cg.gam + (it % 3) * cap, cg.gam + ((it + 2) % 3) * cap, cg.rr + (it % 2) * cap,
                            cg.bbp};
    sum_partials<T, 4>(pr, nparts, tot);
    const T* const pd[1] = {cg.del};
    sum_partials<T, 1>(pd, ndel, dtot);
  }
  const T gi = tot[0], gprev = tot[1], di = dtot[0], rri = tot[2], bb = tot[3];
  const T thresh = cg.tol2 * bb;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cg.res->rr = rri;
    cg.res->bb = bb;
    cg.res->thresh = thresh;
    cg.res->it_last = it;
  }
  if (rri <= thresh || !(rri == rri)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg.res->it = it;
      *cg.done_gen = id;
    }
    return;
  }
  T beta = T(0.0), alpha;
  if (it == 0) {
    alpha = gi / di;
  } else {
    beta = gi / gprev;
    alpha = gi / (di - beta * gi / cg.alpha[(it + 1) % 2]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cg.alpha[it % 2] = alpha;
  T a[2] = {T(0.0), T(0.0)};
  const long lb = xcd_block(blockIdx.x, gridDim.x);
  const long i0 = lb * n / gridDim.x, i1 = (lb + 1) * n / gridDim.x;
  // x is updated every second iteration, with both steps at once:
  // x += alpha_{it-1} p_{it-1} + alpha_it p_it (p_{it-1} is read anyway);
  // k_cg_fix_iso adds a last pending step after the loop.
  const bool odd = (it & 1) != 0;
  const T aprev = odd ? cg.alpha[(it + 1) % 2] : T(0.0);
  // conservation: sum M p by component, as sum s (s = A p, and the SIPG part
  // of A sums to zero)
  CompSum<T> cs;
  cs.init(cg.vs);
  for (long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const T ig = idg[i % NP];
    const T r0 = cg.r[i], wi = cg.w[i];
    const T z0 = ZS ? cg.zs[i] : r0 * ig;  // stored z of the block-Jacobi preconditioner
    const T pold = it == 0 ? T(0.0) : cg.p[i];
    const T pi = z0 + beta * pold;
    const T si = it == 0 ? wi : wi + beta * cg.s[i];
    cg.p[i] = pi;
    cg.s[i] = si;
    if (odd) cg.x[i] = (it == 1 && cg.x0 ? cg.x0[i] : cg.x[i]) + aprev * pold + alpha * pi;
    const T ri = r0 - alpha * si;
    cg.r[i] = ri;
    const T zi = ri * ig;
    a[0] += ri * zi;
    a[1] += ri * ri;
    if (CONS) cs.add(i, cg.vs, si);
  }
  T* const pp[2] = {cg.gam + ((it + 1) % 3) * cap, cg.rr + ((it + 1) % 2) * cap};
  block_partials<T, 2>(a, pp);
  if (CONS) {
    // this block's share of alpha_it sum M p_it joins its running total (the
    // block owns its slots, so no other block reads or writes them)
    cs.fold();
    T tot[kMaxComp];
    block_sum<T, kMaxComp>(cs.acc, tot);
    if (threadIdx.x == 0)
      for (int c = 0; c < kMaxComp; ++c) cg.cons[(10 + c) * cap + blockIdx.x] += alpha * tot[c];
  }
}

// Element-block Jacobi preconditioner of the isotropic operator by fast
// diagonalisation: z_e = A_ee^-1 r_e, A_ee the element's diagonal block of
// M + dt_m K_{nu I}, which on an affine hexahedron (quadrilateral) with
// constant nu is the Kronecker sum J (W x W x W + dtk sum_d K_d x W x W),
// each K_d the one-axis matrix of the host's fds_axis.  With S_d^T W S_d =
// I and S_d^T K_d S_d = diag(lam_d):
//   A_ee^-1 = (1/J) (S_z x S_y x S_x) diag(1 / (1 + dtk (lam_x + lam_y +
//   lam_z))) (S_z x S_y x S_x)^T,
// applied as one contraction per axis forward (S^T), the diagonal, and one
// per axis back (S), through two LDS buffers.  fds: S_0, S_1, S_2 (n1^2
// each, row-major S[i n1 + k]) then lam_0, lam_1, lam_2 (n1 each).  A
// workgroup holds EPB elements of one component (a tile, one thread per
// node) and loops over the (component, tile) pairs of its contiguous range.
// part_rz / part_rr != NULL: block partials of (r, z) and (r, r);
// done_gen != NULL: exit when *done_gen == id.
template <typename T, int DIM, int P>
__global__ void __launch_bounds__((EL<DIM, P>::NT))
k_fds_apply(const T* __restrict__ r, T* __restrict__ z, int nv, Geo g, const T* __restrict__ fds, T dtk,
            T* part_rz, T* part_rr, const int* __restrict__ done_gen, int id) {
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, EPB = L::EPB;
  if (done_gen != nullptr && *done_gen == id) return;
  __shared__ T sS[3 * N1 * N1], sl[3 * N1];
  __shared__ T b0[EPB * NP], b1[EPB * NP];
  for (int k = threadIdx.x; k < 3 * N1 * N1; k += blockDim.x) sS[k] = fds[k];
  for (int k = threadIdx.x; k < 3 * N1; k += blockDim.x) sl[k] = fds[3 * N1 * N1 + k];
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  int ii[3];
  decomp<DIM, N1>(n, ii);
  const int tiles = (g.E + EPB - 1) / EPB, ntot = nv * tiles;
  int t0, t1;
  tile_range(ntot, t0, t1);
  const long vs = (long)g.E * NP;
  const T invJ = T(1.0) / (T)g.J;
  T arz = T(0.0), arr = T(0.0);
  __syncthreads();
  for (int tt = t0; tt < t1; ++tt) {
    const int c = tt / tiles, tile = tt - c * tiles;
    const int e = tile * EPB + le;
    const bool act = le < EPB && e < g.E;
    const long gi = c * vs + (long)e * NP + n;
    const T rv = act ? r[gi] : T(0.0);
    T* const B0 = &b0[le * NP];
    T* const B1 = &b1[le * NP];
    if (le < EPB) B0[n] = rv;
    __syncthreads();
    // forward: u <- S_d^T u along each axis d (B0 -> B1 -> B0 -> B1)
    T* src = B0;
    T* dst = B1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (le < EPB) {
        const int st = L::stride(d);
        const T* row = &src[n - ii[d] * st];
        const T* Sd = &sS[d * N1 * N1];
        T v = T(0.0);
#pragma unroll
        for (int a = 0; a < N1; ++a) v += Sd[a * N1 + ii[d]] * row[a * st];
        dst[n] = v;
      }
      __syncthreads();
      T* tmp = src;
      src = dst;
      dst = tmp;
    }
    if (le < EPB) {
      T lsum = T(0.0);
#pragma unroll
      for (int d = 0; d < DIM; ++d) lsum += sl[d * N1 + ii[d]];
      src[n] *= invJ / (T(1.0) + dtk * lsum);
    }
    __syncthreads();
    // back: u <- S_d u along each axis
#pragma unroll
    for (int d = DIM - 1; d >= 0; --d) {
      if (le < EPB) {
        const int st = L::stride(d);
        const T* row = &src[n - ii[d] * st];
        const T* Sd = &sS[d * N1 * N1];
        T v = T(0.0);
#pragma unroll
        for (int k = 0; k < N1; ++k) v += Sd[ii[d] * N1 + k] * row[k * st];
        dst[n] = v;
      }
      __syncthreads();
      T* tmp = src;
      src = dst;
      dst = tmp;
    }
    if (act) {
      const T zv = src[n];
      z[gi] = zv;
      arz += rv * zv;
      arr += rv * rv;
    }
    __syncthreads();  // the next tile overwrites both buffers
  }
  if (part_rz != nullptr) {
    const T v2[2] = {arz, arr};
    T* const pp[2] = {part_rz, part_rr};
    block_partials<T, 2>(v2, pp);
  }
}

// After the loop of k_cg_iter_iso: if the last iteration that updated the
// vectors (L) was even, x still lacks alpha_L p_L; add it.  L is read from
// the result record (the converged iteration - 1, else the last launched).
// With cg.x0 set, x has not been written before iteration 1: L = 0 adds the
// step to x0, and L < 0 (no update at all) copies x0.
// With cg.cons set, every component is also shifted by the constant that
// makes its total sum M x equal sum b: sum M x = sum M x0 + sum_k alpha_k
// sum M p_k, sum M x0 = sum A x0 (the SIPG part sums to zero), all from the
// partial sums of the start and update kernels, so x is read and written
// once more and nothing else.
template <typename T>
__global__ void k_cg_fix_iso(CGStateT<T> cg, long n, int id) {
  const bool done = *cg.done_gen == id;
  const int L = done ? cg.res->it - 1 : cg.res->it_last;
  T shift[kMaxComp];
#pragma unroll
  for (int c = 0; c < kMaxComp; ++c) shift[c] = T(0.0);
  if (cg.cons) {  // uniform over the grid
    const int cap = cg.cap;
    T sb[kMaxComp], sw[kMaxComp], sp[kMaxComp];
    const T* const pb[kMaxComp] = {cg.cons, cg.cons + cap, cg.cons + 2 * cap, cg.cons + 3 * cap, cg.cons + 4 * cap};
    sum_partials<T, kMaxComp>(pb, cg.nparts, sb);
    const T* const pw[kMaxComp] = {cg.cons + 5 * cap, cg.cons + 6 * cap, cg.cons + 7 * cap, cg.cons + 8 * cap,
                                   cg.cons + 9 * cap};
    sum_partials<T, kMaxComp>(pw, cg.nparts, sw);
    const T* const pr[kMaxComp] = {cg.cons + 10 * cap, cg.cons + 11 * cap, cg.cons + 12 * cap, cg.cons + 13 * cap,
                                   cg.cons + 14 * cap};
    sum_partials<T, kMaxComp>(pr, cg.nparts, sp);
    for (int c = 0; c < cg.nv && c < kMaxComp; ++c) shift[c] = (sb[c] - (sw[c] + sp[c])) / cg.mass_total;
  } else {
    if (L >= 0 && (L & 1)) return;  // x already holds every step (the test is on L >= 0: -1 & 1 is 1)
    if (L < 0 && !cg.x0) return;
  }
  const bool pend = L >= 0 && (L & 1) == 0;  // alpha_L p_L not yet in x
  const T al = pend ? cg.alpha[L % 2] : T(0.0);
  const T* const xs = cg.x0 && L <= 0 ? cg.x0 : cg.x;  // x0 when x was never written (no odd update)
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    T v = xs[i];
    if (pend) v += al * cg.p[i];
    if (cg.cons) {
      const int c = (int)(i / cg.vs);
#pragma unroll
      for (int k = 0; k < kMaxComp; ++k)
        if (k == c) v += shift[k];
    }
    cg.x[i] = v;
  }
}

// Jacobi diagonal of M + dt_m K_D (volume terms with d = d' and the face
// terms of the node itself); any positive diagonal gives the same solution.
template <typename T, int DIM, int P>
__global__ void __launch_bounds__((EL<DIM, P>::NT))
k_helm_diag(T* __restrict__ diag, int nv, long vs, CoefT<T> cf, T dtm, T ctau, Geo g,
            const T* __restrict__ tab) {
  const T rh2[3] = {(T)g.rh2[0], (T)g.rh2[1], (T)g.rh2[2]};
  const T gJ = (T)g.J;
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, EPB = L::EPB;
  __shared__ T sD[N1 * N1], sw[N1];
  __shared__ T sc[EPB * NP];
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  const int e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool act = (le < EPB) && (e < g.E);
  for (int k = t; k < N1 * N1; k += blockDim.x) sD[k] = tab[k];
  for (int k = t; k < N1; k += blockDim.x) sw[k] = tab[N1 * N1 + k];
  int ii[3];
  decomp<DIM, N1>(n, ii);
  const long own = (long)e * NP + n;
  if (act) sc[le * NP + n] = coef_w2(cf, own);
  __syncthreads();
  if (!act) return;
  T wn = T(1.0);
  for (int d = 0; d < DIM; ++d) wn *= sw[ii[d]];
  const T nue = coef_nu(cf, e);
  T kd = T(0.0);
  for (int d = 0; d < DIM; ++d) {
    const int st = L::stride(d);
    T s = T(0.0);
    for (int k = 0; k < N1; ++k) {
      const int nk = n + (k - ii[d]) * st;
      const T dd = sc[le * NP + nk] * cf.v[d] * cf.v[d] + nue;
      const T wk = wn / sw[ii[d]] * sw[k];
      s += sD[k * N1 + ii[d]] * sD[k * N1 + ii[d]] * wk * dd;
    }
    kd += rh2[d] * rh2[d] * gJ * s;
  }
  const T dow_c = sc[le * NP + n];
  for (int d = 0; d < DIM; ++d) {
    for (int side = 0; side < 2; ++side) {
      if (ii[d] != (side ? P : 0)) continue;
      const T sgn = side ? T(1.0) : -T(1.0);
      const int nb = neighbour(g, e, d, side ? 1 : -1);
      const int nn = n + ((side ? 0 : P) - ii[d]) * L::stride(d);
      const T dnb = coef_w2(cf, (long)nb * NP + nn) * cf.v[d] * cf.v[d] + coef_nu(cf, nb);
      const T dow = dow_c * cf.v[d] * cf.v[d] + nue;
      const T tau = ctau * (T)(N1 * N1) * fmax(dow, dnb) * T(0.5) * rh2[d];
      const T jfwf = gJ * rh2[d] * wn / sw[ii[d]];
      kd += jfwf * (tau - sgn * rh2[d] * dow * sD[ii[d] * N1 + ii[d]]);
    }
  }
  const T val = gJ * wn + dtm * kd;
  for (int c = 0; c < nv; ++c) diag[c * vs + own] = val;
}

// ---------------------------------------------------------------- PCG
// Chronopoulos-Gear form of Jacobi-PCG: per iteration one element kernel
// (vector updates, z = diag^-1 r, face traces of z, partials of (r,z) and
// (r,r)) and one matvec kernel (w = A z with the partial of (w,z)):
//   beta_i = g_i / g_{i-1},  alpha_i = g_i / (d_i - beta_i g_i / alpha_{i-1})
//   p = z + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   z = r / diag,  w = A z,  g = (r, z),  d = (w, z).
//
// Start: r = b - A x0 (A x0 given in w), z = r / diag, traces of z; partials
// (r,z) -> gam[0], (r,r) -> rr[0], (b,b) -> bbp.
template <typename T, int DIM, int P>
__global__ void __launch_bounds__((EL<DIM, P>::NT))
k_cg_start(CGStateT<T> cg, int nv, long vs, CoefT<T> cf, Geo g, const T* __restrict__ tab) {
  const T rh2[3] = {(T)g.rh2[0], (T)g.rh2[1], (T)g.rh2[2]};
  const T gJ = (T)g.J;
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, EPB = L::EPB;
  __shared__ T sD[N1 * N1];
  __shared__ T sx[EPB * NP];
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  for (int k = t; k < N1 * N1; k += blockDim.x) sD[k] = tab[k];
  int ii[3];
  decomp<DIM, N1>(n, ii);
  const int ntiles = (g.E + EPB - 1) / EPB;
  T a[3] = {T(0.0), T(0.0), T(0.0)};
  int tile0, tile1;
  tile_range(ntiles, tile0, tile1);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int e = tile * EPB + le;
    const bool act = (le < EPB) && (e < g.E);
    const long own = (long)e * NP + n;
    const T cw = act ? coef_w2(cf, own) : T(0.0);
    for (int c = 0; c < nv; ++c) {
      const long i = c * vs + own;
      __syncthreads();
      if (act) {
        const T bi = cg.b[i];
        const T ri = bi - cg.w[i];
        const T zi = ri / cg.diag[i];
        cg.r[i] = ri;
        cg.z[i] = zi;
        sx[le * NP + n] = zi;
        a[0] += ri * zi;
        a[1] += ri * ri;
        a[2] += bi * bi;
      }
      __syncthreads();
      if (act) store_trace<T, DIM, P>(&sx[le * NP], sD, n, ii, cw, cf, g, cg.trace, c, e);
    }
  }
  T* const pp[3] = {cg.gam, cg.rr, cg.bbp};
  block_partials<T, 3>(a, pp);
}

// Iteration `it` of the element part.  Reads the partials of g_it (gam[it%3]),
// g_{it-1}, d_it (del), (r,r)_it (rr[it%2]); stops the solve if
// (r,r)_it <= rtol^2 (b,b); otherwise updates p, s, x, r, z, writes the face
// traces of the new z and the partials of g_{it+1} and (r,r)_{it+1}.
template <typename T, int DIM, int P>
__global__ void __launch_bounds__((EL<DIM, P>::NT))
k_cg_iter(CGStateT<T> cg, int nv, long vs, CoefT<T> cf, Geo g, const T* __restrict__ tab, int it, int id,
          int nparts) {
  const T rh2[3] = {(T)g.rh2[0], (T)g.rh2[1], (T)g.rh2[2]};
  const T gJ = (T)g.J;
  using L = EL<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, EPB = L::EPB;
  if (*cg.done_gen == id) return;
  __shared__ T sD[N1 * N1];
  __shared__ T sx[EPB * NP];
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  for (int k = t; k < N1 * N1; k += blockDim.x) sD[k] = tab[k];
  int ii[3];
  decomp<DIM, N1>(n, ii);
  const int cap = cg.cap;
  T tot[5];
  {
    const T* const pr[5] = {cg.gam + (it % 3) * cap, cg.gam + ((it + 2) % 3) * cap, cg.del,
                                 cg.rr + (it % 2) * cap, cg.bbp};
    sum_partials<T, 5>(pr, nparts, tot);
  }
  const T gi = tot[0], gprev = tot[1], di = tot[2], rri = tot[3], bb = tot[4];
  const T thresh = cg.tol2 * bb;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cg.res->rr = rri;
    cg.res->bb = bb;
    cg.res->thresh = thresh;
    cg.res->it_last = it;
  }
  if (rri <= thresh || !(rri == rri)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg.res->it = it;
      *cg.done_gen = id;
    }
    return;
  }
  T beta = T(0.0), alpha;
  if (it == 0) {
    alpha = gi / di;
  } else {
    beta = gi / gprev;
    alpha = gi / (di - beta * gi / cg.alpha[(it + 1) % 2]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cg.alpha[it % 2] = alpha;
  const int ntiles = (g.E + EPB - 1) / EPB;
  T a[2] = {T(0.0), T(0.0)};
  int tile0, tile1;
  tile_range(ntiles, tile0, tile1);
  for (int tile = tile0; tile < tile1; ++tile) {
    const int e = tile * EPB + le;
    const bool act = (le < EPB) && (e < g.E);
    const long own = (long)e * NP + n;
    const T cw = act ? coef_w2(cf, own) : T(0.0);
    for (int c = 0; c < nv; ++c) {
      const long i = c * vs + own;
      __syncthreads();
      if (act) {
        const T zi0 = cg.z[i], wi = cg.w[i];
        const T pi = it == 0 ? zi0 : zi0 + beta * cg.p[i];
        const T si = it == 0 ? wi : wi + beta * cg.s[i];
        cg.p[i] = pi;
        cg.s[i] = si;
        cg.x[i] += alpha * pi;
        const T ri = cg.r[i] - alpha * si;
        const T zi = ri / cg.diag[i];
        cg.r[i] = ri;
        cg.z[i] = zi;
        sx[le * NP + n] = zi;
        a[0] += ri * zi;
        a[1] += ri * ri;
      }
      __syncthreads();
      if (act) store_trace<T, DIM, P>(&sx[le * NP], sD, n, ii, cw, cf, g, cg.trace, c, e);
    }
  }
  T* const pp[2] = {cg.gam + ((it + 1) % 3) * cap, cg.rr + ((it + 1) % 2) * cap};
  block_partials<T, 2>(a, pp);
}

// ---------------------------------------------------------------- vectors
__global__ void k_lincomb(double* __restrict__ out, LinComb lc, long n, const double* __restrict__ mw,
                          int np) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double m = mw[i % np];
    double s = 0.0;
    for (int j = 0; j < lc.n; ++j) s += lc.c[j] * (lc.m[j] ? m : 1.0) * lc.x[j][i];
    out[i] = s;
  }
}

// One axis of a tensor-product transfer on an LDS grid: dst = A along axis
// `ax` of src (n0 x n1 x n2, axis 0 fastest), A an (m x n_ax) row-major
// matrix; dst is the same grid with n_ax replaced by m.
__device__ void contract_axis(const double* src, double* dst, const double* A, int ax, int n0, int n1, int n2,
                              int m) {
  const int na = ax == 0 ? n0 : (ax == 1 ? n1 : n2);
  const int o0 = ax == 0 ? m : n0, o1 = ax == 1 ? m : n1, o2 = ax == 2 ? m : n2;
  const int tot = o0 * o1 * o2;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int i0 = idx % o0, i1 = (idx / o0) % o1, i2 = idx / (o0 * o1);
    const int r = ax == 0 ? i0 : (ax == 1 ? i1 : i2);
    double acc = 0.0;
    for (int a = 0; a < na; ++a) {
      const int j0 = ax == 0 ? a : i0, j1 = ax == 1 ? a : i1, j2 = ax == 2 ? a : i2;
      acc += A[r * na + a] * src[(j2 * n1 + j1) * n0 + j0];
    }
    dst[idx] = acc;
  }
}

// 2:1 h-coarsening transfer (p-coarsening on top): one block per (variable,
// coarse element).  A is the 1-D matrix on an axis' pair of fine elements
// (2 n1f nodes, left child first), applied along every axis:
//   mode 0, fine -> coarse: A is (n1c x 2 n1f); the input is the 2^dim children
//   mode 1, coarse -> fine: A is (2 n1f x n1c); the output is the 2^dim children
// Fine element (2 cx + kx, 2 cy + ky, 2 cz + kz) is child (kx, ky, kz) of
// coarse element (cx, cy, cz); its node i along an axis is node k n1f + i of
// the pair.  The grid of a pair fits kHGrid doubles: (2 n1f)^dim <= kHGrid.
constexpr int kHGrid = 2744;
__global__ void k_space_transfer_h(const double* __restrict__ in, double* __restrict__ out, int dim, int n1f, int n1c,
                                   int ncx, int ncy, int ncz, const double* __restrict__ A, int mode) {
  __shared__ double sa[kHGrid], sb[kHGrid];
  __shared__ double sA[2 * (kMaxP + 1) * (kMaxP + 1)];
  const int Ec = ncx * ncy * ncz;
  const int nfx = 2 * ncx, nfy = 2 * ncy;
  const long Ef = (long)Ec << dim;
  const int var = (int)(blockIdx.x / Ec), ec = (int)(blockIdx.x % Ec);
  const int cx = ec % ncx, cy = (ec / ncx) % ncy, cz = ec / (ncx * ncy);
  const int S = 2 * n1f;
  const int ni = mode == 0 ? S : n1c, no = mode == 0 ? n1c : S;
  const int npf = dim == 2 ? n1f * n1f : n1f * n1f * n1f;
  const int npc = dim == 2 ? n1c * n1c : n1c * n1c * n1c;
  for (int k = threadIdx.x; k < no * ni; k += blockDim.x) sA[k] = A[k];
  const int nin = dim == 2 ? ni * ni : ni * ni * ni;
  for (int idx = threadIdx.x; idx < nin; idx += blockDim.x) {
    if (mode == 0) {
      const int X = idx % ni, Y = (idx / ni) % ni, Z = dim == 3 ? idx / (ni * ni) : 0;
      const int kx = X / n1f, ky = Y / n1f, kz = Z / n1f;
      const int ix = X - kx * n1f, iy = Y - ky * n1f, iz = Z - kz * n1f;
      const long fe = (2 * cx + kx) + (long)nfx * ((2 * cy + ky) + (long)nfy * (2 * cz + kz));
      const int node = ix + n1f * (iy + n1f * iz);
      sa[idx] = in[((long)var * Ef + fe) * npf + node];
    } else {
      sa[idx] = in[((long)var * Ec + ec) * npc + idx];
    }
  }
  __syncthreads();
  const int n2 = dim == 3 ? ni : 1;
  contract_axis(sa, sb, sA, 0, ni, ni, n2, no);
  __syncthreads();
  contract_axis(sb, sa, sA, 1, no, ni, n2, no);
  __syncthreads();
  const double* res = sa;
  if (dim == 3) {
    contract_axis(sa, sb, sA, 2, no, no, ni, no);
    __syncthreads();
    res = sb;
  }
  const int nout = dim == 2 ? no * no : no * no * no;
  for (int idx = threadIdx.x; idx < nout; idx += blockDim.x) {
    if (mode == 0) {
      out[((long)var * Ec + ec) * npc + idx] = res[idx];
    } else {
      const int X = idx % no, Y = (idx / no) % no, Z = dim == 3 ? idx / (no * no) : 0;
      const int kx = X / n1f, ky = Y / n1f, kz = Z / n1f;
      const int ix = X - kx * n1f, iy = Y - ky * n1f, iz = Z - kz * n1f;
      const long fe = (2 * cx + kx) + (long)nfx * ((2 * cy + ky) + (long)nfy * (2 * cz + kz));
      const int node = ix + n1f * (iy + n1f * iz);
      out[((long)var * Ef + fe) * npf + node] = res[idx];
    }
  }
}

// Several combinations of the same vectors in one pass: each input is read
// once (the node quadrature q_m = sum_i S_{m,i} f_i for all m at once).
__global__ void k_lincomb_multi(double* __restrict__ out, LinCombMulti lc, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double xv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) xv[j] = j < lc.nin ? lc.x[j][i] : 0.0;
    for (int o = 0; o < lc.nout; ++o) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < lc.nin) s += lc.c[o][j] * xv[j];
      out[(long)o * n + i] = s;
    }
  }
}

// Collocation residual of all nodes in one pass over u, f (and g).
__global__ void k_colloc_residual(CollocResid c, long n, const double* __restrict__ mw, int np) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double w = mw[i % np];
    double fv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) fv[j] = j < c.M ? c.f[(long)j * n + i] : 0.0;
    double prev = c.u[i];
    for (int m = 1; m <= c.M; ++m) {
      const double cur = c.u[(long)m * n + i];
      double q = 0.0;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < c.M) q += c.S[m - 1][j] * fv[j];
      double r = c.sign * (w * (cur - prev) - q);
      if (c.g) r += c.g[(long)(m - 1) * n + i];
      c.out[(long)(m - 1) * n + i] = r;
      prev = cur;
    }
  }
}

// out[var][e][o] = sum_{a,b,c} A[ox][a] A[oy][b] A[oz][c] in[var][e][(a,b,c)]
// Output node o of the tensor-product map (A x A [x A]) applied to one
// element's nodal values sin_ (n1i per direction, x fastest).
__device__ __forceinline__ double tp_map(const double* sA, const double* sin_, int o, int dim, int n1i, int n1o) {
  const int ox = o % n1o, oy = (o / n1o) % n1o, oz = dim == 3 ? o / (n1o * n1o) : 0;
  double s = 0.0;
  if (dim == 2) {
    for (int b = 0; b < n1i; ++b) {
      double t = 0.0;
      for (int a = 0; a < n1i; ++a) t += sA[ox * n1i + a] * sin_[b * n1i + a];
      s += sA[oy * n1i + b] * t;
    }
  } else {
    for (int c = 0; c < n1i; ++c) {
      double tc = 0.0;
      for (int b = 0; b < n1i; ++b) {
        double t = 0.0;
        for (int a = 0; a < n1i; ++a) t += sA[ox * n1i + a] * sin_[(c * n1i + b) * n1i + a];
        tc += sA[oy * n1i + b] * t;
      }
      s += sA[oz * n1i + c] * tc;
    }
  }
  return s;
}

__global__ void k_space_transfer(const double* __restrict__ in, double* __restrict__ out, int dim,
                                 int n1i, int n1o, int E, const double* __restrict__ A) {
  __shared__ double sA[(kMaxP + 1) * (kMaxP + 1)];
  __shared__ double sin_[(kMaxP + 1) * (kMaxP + 1) * (kMaxP + 1)];
  const int npi = dim == 2 ? n1i * n1i : n1i * n1i * n1i;
  const int npo = dim == 2 ? n1o * n1o : n1o * n1o * n1o;
  const long blk = blockIdx.x;  // (var, e)
  for (int k = threadIdx.x; k < n1i * n1o; k += blockDim.x) sA[k] = A[k];
  for (int k = threadIdx.x; k < npi; k += blockDim.x) sin_[k] = in[blk * npi + k];
  __syncthreads();
  for (int o = threadIdx.x; o < npo; o += blockDim.x) out[blk * npo + o] = tp_map(sA, sin_, o, dim, n1i, n1o);
}

// Space-time transfer, one block per (component, element): every source
// vector of the element is read once, the time combinations of all output
// nodes are formed in LDS, then each output node is mapped in space by sum
// factorisation (one 1-D contraction per axis, through two LDS buffers).
// Inputs and outputs belong to levels with the same elements.  Dynamic LDS:
// A (n1o x n1i), nout * npi time combinations, two buffers of n1max^dim.
__global__ void __launch_bounds__(256)
k_space_time_transfer(TransferMulti t, int dim, int n1i, int n1o, const double* __restrict__ A) {
  extern __shared__ double smem[];
  const int npi = dim == 2 ? n1i * n1i : n1i * n1i * n1i;
  const int npo = dim == 2 ? n1o * n1o : n1o * n1o * n1o;
  const int n1m = n1i > n1o ? n1i : n1o;
  const int nbuf = dim == 2 ? n1m * n1m : n1m * n1m * n1m;
  double* const sA = smem;                 // A[o * n1i + i]
  double* const sT = sA + n1o * n1i;       // time combinations, nout x npi
  double* const sB0 = sT + t.nout * npi;
  double* const sB1 = sB0 + nbuf;
  const long blk = blockIdx.x;  // (component, element)
  for (int k = threadIdx.x; k < n1i * n1o; k += blockDim.x) sA[k] = A[k];
  for (int k = threadIdx.x; k < npi; k += blockDim.x) {
    double xv[kTransferIn];
#pragma unroll
    for (int j = 0; j < kTransferIn; ++j) xv[j] = j < t.nin ? t.x[j][blk * npi + k] : 0.0;
    for (int mo = 0; mo < t.nout; ++mo) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < kTransferIn; ++j) v += t.c[mo][j] * xv[j];
      sT[mo * npi + k] = v;
    }
  }
  __syncthreads();
  for (int mo = 0; mo < t.nout; ++mo) {
    const double* const src = sT + mo * npi;
    double* const y = t.y[mo];
    double* const y2 = t.y2[mo];
    if (dim == 3) {
      // x: B0[(c n1i + b) n1o + ox] = sum_a A[ox][a] src[(c n1i + b) n1i + a]
      for (int k = threadIdx.x; k < n1i * n1i * n1o; k += blockDim.x) {
        const int ox = k % n1o, cb = k / n1o;
        double v = 0.0;
        for (int a = 0; a < n1i; ++a) v += sA[ox * n1i + a] * src[cb * n1i + a];
        sB0[k] = v;
      }
      __syncthreads();
      // y: B1[(c n1o + oy) n1o + ox] = sum_b A[oy][b] B0[(c n1i + b) n1o + ox]
      for (int k = threadIdx.x; k < n1i * n1o * n1o; k += blockDim.x) {
        const int ox = k % n1o, oy = (k / n1o) % n1o, c = k / (n1o * n1o);
        double v = 0.0;
        for (int b = 0; b < n1i; ++b) v += sA[oy * n1i + b] * sB0[(c * n1i + b) * n1o + ox];
        sB1[k] = v;
      }
      __syncthreads();
      // z: out[(oz n1o + oy) n1o + ox] = sum_c A[oz][c] B1[(c n1o + oy) n1o + ox]
      for (int o = threadIdx.x; o < npo; o += blockDim.x) {
        const int oxy = o % (n1o * n1o), oz = o / (n1o * n1o);
        double v = 0.0;
        for (int c = 0; c < n1i; ++c) v += sA[oz * n1i + c] * sB1[c * n1o * n1o + oxy];
        if (t.accumulate) v += y[blk * npo + o];
        y[blk * npo + o] = v;
        if (y2) y2[blk * npo + o] = v;
      }
    } else {
      // x: B0[b n1o + ox] = sum_a A[ox][a] src[b n1i + a]
      for (int k = threadIdx.x; k < n1i * n1o; k += blockDim.x) {
        const int ox = k % n1o, b = k / n1o;
        double v = 0.0;
        for (int a = 0; a < n1i; ++a) v += sA[ox * n1i + a] * src[b * n1i + a];
        sB0[k] = v;
      }
      __syncthreads();
      for (int o = threadIdx.x; o < npo; o += blockDim.x) {
        const int ox = o % n1o, oy = o / n1o;
        double v = 0.0;
        for (int b = 0; b < n1i; ++b) v += sA[oy * n1i + b] * sB0[b * n1o + ox];
        if (t.accumulate) v += y[blk * npo + o];
        y[blk * npo + o] = v;
        if (y2) y2[blk * npo + o] = v;
      }
    }
    __syncthreads();  // the next output node overwrites the buffers
  }
}

// out = in, word by word (device copies of a step under graph capture are
// kernels, not copy nodes)
__global__ void k_copy(const double* __restrict__ in, double* __restrict__ out, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) out[i] = in[i];
}

__global__ void k_cast_f(const double* __restrict__ in, float* __restrict__ out, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// r32 = (float)(b - Ax) with FP64 partial sums of (r,r) and (b,b) per block.
__global__ void k_resid_cast(const double* __restrict__ b, const double* __restrict__ Ax, float* __restrict__ r32,
                             long n, double* part) {
  double a[2] = {0.0, 0.0};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double bi = b[i];
    const double ri = bi - Ax[i];
    r32[i] = (float)ri;
    a[0] += ri * ri;
    a[1] += bi * bi;
  }
  double* const pp[2] = {part, part + kElemCap};
  block_partials<double, 2>(a, pp);
}

// tot[0..1] = fixed-order sums of the n partials in part and part + kElemCap.
__global__ void k_sum2(const double* __restrict__ part, int n, double* tot) {
  const double* const pp[2] = {part, part + kElemCap};
  double t[2];
  sum_partials<double, 2>(pp, n, t);
  if (threadIdx.x == 0) {
    tot[0] = t[0];
    tot[1] = t[1];
  }
}

// block partials of (a, b) -> part[blk] and (a, c) -> part[kElemCap + blk]
// Conservation correction of an implicit solve (A = M + dt_m K_D, K_D
// symmetric with the constants in its kernel, so 1^T A x = 1^T M x): per
// component c, x_c += (1^T b_c - 1^T M x_c) / 1^T M 1, which makes the
// solution's total 1^T M x equal the right-hand side's total up to the
// rounding of the sums.  b is a vector or, when b == NULL, the combination
// lc (mass weights where lc.m[j]).  Pass 1: grid (nb, nv), block partials of
// both sums per component into part[(2 c) nb + blk] and part[(2 c + 1) nb +
// blk]; pass 2: grid (*, nv), every block sums its component's partials in
// the same fixed order and adds the constant.
__global__ void k_conserve_sums(const double* __restrict__ b, LinComb lc, const double* __restrict__ x, long vs,
                                const double* __restrict__ mw, int np, double* part) {
  const int c = blockIdx.y, nb = gridDim.x;
  const long o = (long)c * vs;
  double v[2] = {0.0, 0.0};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < vs; i += (long)nb * blockDim.x) {
    const double m = mw[i % np];
    double bi;
    if (b) {
      bi = b[o + i];
    } else {
      bi = 0.0;
      for (int j = 0; j < lc.n; ++j) bi += lc.c[j] * (lc.m[j] ? m : 1.0) * lc.x[j][o + i];
    }
    v[0] += bi;
    v[1] += m * x[o + i];
  }
  double* const pp[2] = {part + (long)(2 * c) * nb, part + (long)(2 * c + 1) * nb};
  block_partials<double, 2>(v, pp);
}

__global__ void k_conserve_apply(double* __restrict__ x, long vs, const double* __restrict__ part, int nb,
                                 double mass_total) {
  const int c = blockIdx.y;
  double tot[2];
  const double* const pr[2] = {part + (long)(2 * c) * nb, part + (long)(2 * c + 1) * nb};
  sum_partials<double, 2>(pr, nb, tot);
  const double shift = (tot[0] - tot[1]) / mass_total;
  double* const xc = x + (long)c * vs;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < vs; i += (long)gridDim.x * blockDim.x) xc[i] += shift;
}

__global__ void k_dot2(const double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ c,
                       long n, double* part) {
  double v[2] = {0.0, 0.0};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    v[0] += a[i] * b[i];
    v[1] += a[i] * c[i];
  }
  double* const pp[2] = {part, part + kElemCap};
  block_partials<double, 2>(v, pp);
}

// x += (double) e
__global__ void k_add_f2d(double* __restrict__ x, const float* __restrict__ e, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] += (double)e[i];
}

// Per-block maxima of max_d (|v_d| + c) and minima of rho (Euler /
// Navier-Stokes) into part[b] and part[kElemCap + b]; reduced by
// k_maxmin_partials.
template <int DIM>
__global__ void k_euler_lam(const double* __restrict__ u, long vs, EqP q, double* part) {
  constexpr int NV = DIM + 2;
  __shared__ double sm[16], sr[16];
  double m = 0.0, rmin = 1e300;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < vs; i += (long)gridDim.x * blockDim.x) {
    double uu[NV];
    for (int v = 0; v < NV; ++v) uu[v] = u[v * vs + i];
    for (int d = 0; d < DIM; ++d) m = fmax(m, wave_speed<NV>(q, d, uu));
    rmin = fmin(rmin, uu[0]);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    m = fmax(m, __shfl_down(m, off, 64));
    rmin = fmin(rmin, __shfl_down(rmin, off, 64));
  }
  if (lane == 0) {
    sm[wid] = m;
    sr[wid] = rmin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, r = 1e300;
    for (int w = 0; w < nw; ++w) {
      s = fmax(s, sm[w]);
      r = fmin(r, sr[w]);
    }
    part[blockIdx.x] = s;
    part[kElemCap + blockIdx.x] = r;
  }
}

__global__ void k_maxmin_partials(const double* __restrict__ part, int n, double* result) {
  __shared__ double sm[16], sr[16];
  double m = 0.0, rmin = 1e300;
  for (int b = threadIdx.x; b < n; b += blockDim.x) {
    m = fmax(m, part[b]);
    rmin = fmin(rmin, part[kElemCap + b]);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    m = fmax(m, __shfl_down(m, off, 64));
    rmin = fmin(rmin, __shfl_down(rmin, off, 64));
  }
  if (lane == 0) {
    sm[wid] = m;
    sr[wid] = rmin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, r = 1e300;
    for (int w = 0; w < nw; ++w) {
      s = fmax(s, sm[w]);
      r = fmin(r, sr[w]);
    }
    result[0] = s;
    result[1] = r;
  }
}

// ---------------------------------------------------------------- launchers
static inline int blocks_for(long n, int bs, int cap) {
  long b = (n + bs - 1) / bs;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

template <int DIM, int P>
static int elem_tiles(const Geo& g) {
  return (g.E + EL<DIM, P>::EPB - 1) / EL<DIM, P>::EPB;
}

int elem_tile_count(const Geo& g) {
  const int epb = g.np >= 256 ? 1 : 256 / g.np;
  return (g.E + epb - 1) / epb;
}

int reduce_grid(const Geo& g) { return std::min(elem_tile_count(g), kElemCap); }

#define SISDC_DISPATCH_P(P_, BODY)                   \
  switch (P_) {                                      \
    case 1: { constexpr int PP = 1; BODY; } break;  \
    case 2: { constexpr int PP = 2; BODY; } break;  \
    case 3: { constexpr int PP = 3; BODY; } break;  \
    case 4: { constexpr int PP = 4; BODY; } break;  \
    case 5: { constexpr int PP = 5; BODY; } break;  \
    case 6: { constexpr int PP = 6; BODY; } break;  \
    case 7: { constexpr int PP = 7; BODY; } break;  \
    case 8: { constexpr int PP = 8; BODY; } break;  \
    default: return hipErrorInvalidValue;            \
  }

#define SISDC_DISPATCH(G_, FN, ...)                                                            \
  do {                                                                                         \
    if ((G_).dim == 2) { SISDC_DISPATCH_P((G_).P, return (FN<2, PP>(__VA_ARGS__))); }         \
    else if ((G_).dim == 3) { SISDC_DISPATCH_P((G_).P, return (FN<3, PP>(__VA_ARGS__))); }    \
    return hipErrorInvalidValue;                                                               \
  } while (0)

template <int DIM, int P>
static hipError_t conv_dim_p(const double* u, double* out, const Geo& g, const EqP& q, const double* tab,
                             int nodes, hipStream_t s) {
  using L = EL<DIM, P>;
  const long vs = (long)g.E * L::NP;
  const dim3 grid(elem_tiles<DIM, P>(g), nodes);
  if (nodes < 1)
    return hipErrorInvalidValue;
  else if (q.nv == 1)
    hipLaunchKernelGGL((k_conv<DIM, P, 1>), grid, dim3(L::NTF), 0, s, u, out, g, q, tab, vs);
  else if (q.nv == DIM + 2)
    hipLaunchKernelGGL((k_conv<DIM, P, DIM + 2>), grid, dim3(L::NTF), 0, s, u, out, g, q, tab, vs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_conv(const double* u, double* out, const Geo& g, const EqP& q, const double* tab,
                       hipStream_t s, int nodes) {
  SISDC_DISPATCH(g, conv_dim_p, u, out, g, q, tab, nodes, s);
}

template <typename T, int DIM, int P>
static hipError_t trace_dim_p(const T* x, int nv, const CoefT<T>& cf, T* trace, const Geo& g, const T* tab,
                              hipStream_t s) {
  using L = EL<DIM, P>;
  const long vs = (long)g.E * L::NP;
  hipLaunchKernelGGL((k_sipg_trace<T, DIM, P>), dim3(elem_tiles<DIM, P>(g)), dim3(L::NT), 0, s, x, nv, vs, cf,
                     trace, g, tab);
  return hipGetLastError();
}

template <typename T>
static hipError_t sipg_trace_t(const T* x, int nv, const CoefT<T>& cf, T* trace, const Geo& g, const T* tab,
                               hipStream_t s) {
  if (g.dim == 2) { SISDC_DISPATCH_P(g.P, return (trace_dim_p<T, 2, PP>(x, nv, cf, trace, g, tab, s))); }
  if (g.dim == 3) { SISDC_DISPATCH_P(g.P, return (trace_dim_p<T, 3, PP>(x, nv, cf, trace, g, tab, s))); }
  return hipErrorInvalidValue;
}

// The isotropic hexahedral kernel serves D = nu I (no convective part, no
// coefficient state) for the degrees whose line groups tile a wave.
template <typename T>
static bool iso_coef(const CoefT<T>& cf) {
  return cf.ub == nullptr && cf.eps == nullptr && cf.v[0] == T(0.0) && cf.v[1] == T(0.0) && cf.v[2] == T(0.0);
}

template <typename T, int DIM, int P>
static hipError_t apply_iso_p(const T* x, const T* isc, T* out, int nv, const CoefT<T>& cf, T alpha, T beta,
                              T ctau, const Geo& g, const T* tab, T* part, const int* done_gen, int id,
                              hipStream_t s);

template <typename T, int DIM, int P>
static hipError_t apply_dim_p(const T* x, T* out, int nv, const CoefT<T>& cf, const T* trace, T alpha, T beta,
                              T ctau, const Geo& g, const T* tab, const T* dotv, T* part, const int* done_gen,
                              int id, hipStream_t s) {
  using L = EL<DIM, P>;
  const long vs = (long)g.E * L::NP;
  // the partial count must equal the grid of the CG kernels that sum them
  const int nb = part ? std::min(elem_tiles<DIM, P>(g), kElemCap) : elem_tiles<DIM, P>(g);
  if constexpr (DIM == 2 || P == 1 || P == 3 || P == 7) {
    // the isotropic kernel in the launch configuration of the isotropic CG
    // (launch_sipg_apply_iso), so a stage application runs the same grid
    if (iso_coef(cf) && part == nullptr)
      return apply_iso_p<T, DIM, P>(x, nullptr, out, nv, cf, alpha, beta, ctau, g, tab, nullptr, done_gen, id, s);
  }
  hipLaunchKernelGGL((k_sipg_apply<T, DIM, P>), dim3(nb), dim3(L::NT), 0, s, x, out, nv, vs, cf, trace, alpha,
                     beta, ctau, g, tab, dotv, part, done_gen, id);
  return hipGetLastError();
}

template <typename T>
static hipError_t sipg_apply_t(const T* x, T* out, int nv, const CoefT<T>& cf, const T* trace, T alpha, T beta,
                               T ctau, const Geo& g, const T* tab, const T* dotv, T* part, const int* done_gen,
                               int id, hipStream_t s) {
  if (g.dim == 2) {
    SISDC_DISPATCH_P(g.P, return (apply_dim_p<T, 2, PP>(x, out, nv, cf, trace, alpha, beta, ctau, g, tab, dotv,
                                                         part, done_gen, id, s)));
  }
  if (g.dim == 3) {
    SISDC_DISPATCH_P(g.P, return (apply_dim_p<T, 3, PP>(x, out, nv, cf, trace, alpha, beta, ctau, g, tab, dotv,
                                                         part, done_gen, id, s)));
  }
  return hipErrorInvalidValue;
}

template <typename T, int DIM, int P>
static hipError_t diag_dim_p(T* diag, int nv, const CoefT<T>& cf, T dtm, T ctau, const Geo& g, const T* tab,
                             hipStream_t s, bool first_only = false) {
  using L = EL<DIM, P>;
  const long vs = (long)g.E * L::NP;
  // first_only: one workgroup, i.e. the first EPB elements, component 0
  hipLaunchKernelGGL((k_helm_diag<T, DIM, P>), dim3(first_only ? 1 : elem_tiles<DIM, P>(g)), dim3(L::NT), 0, s, diag,
                     first_only ? 1 : nv, vs, cf, dtm, ctau, g, tab);
  return hipGetLastError();
}

template <typename T>
static hipError_t helm_diag_t(T* diag, int nv, const CoefT<T>& cf, T dtm, T ctau, const Geo& g, const T* tab,
                              hipStream_t s) {
  if (g.dim == 2) { SISDC_DISPATCH_P(g.P, return (diag_dim_p<T, 2, PP>(diag, nv, cf, dtm, ctau, g, tab, s))); }
  if (g.dim == 3) { SISDC_DISPATCH_P(g.P, return (diag_dim_p<T, 3, PP>(diag, nv, cf, dtm, ctau, g, tab, s))); }
  return hipErrorInvalidValue;
}

template <typename T, int DIM, int P>
static hipError_t cg_start_dim_p(const CGStateT<T>& cg, int nv, const CoefT<T>& cf, const Geo& g, const T* tab,
                                 hipStream_t s) {
  using L = EL<DIM, P>;
  const long vs = (long)g.E * L::NP;
  hipLaunchKernelGGL((k_cg_start<T, DIM, P>), dim3(std::min(elem_tiles<DIM, P>(g), kElemCap)), dim3(L::NT), 0, s,
                     cg, nv, vs, cf, g, tab);
  return hipGetLastError();
}

template <typename T>
static hipError_t cg_start_t(const CGStateT<T>& cg, int nv, const CoefT<T>& cf, const Geo& g, const T* tab,
                             hipStream_t s) {
  if (g.dim == 2) { SISDC_DISPATCH_P(g.P, return (cg_start_dim_p<T, 2, PP>(cg, nv, cf, g, tab, s))); }
  if (g.dim == 3) { SISDC_DISPATCH_P(g.P, return (cg_start_dim_p<T, 3, PP>(cg, nv, cf, g, tab, s))); }
  return hipErrorInvalidValue;
}

template <typename T, int DIM, int P>
static hipError_t cg_iter_dim_p(const CGStateT<T>& cg, int nv, const CoefT<T>& cf, const Geo& g, const T* tab,
                                int it, int id, hipStream_t s) {
  using L = EL<DIM, P>;
  const long vs = (long)g.E * L::NP;
  const int nb = std::min(elem_tiles<DIM, P>(g), kElemCap);
  hipLaunchKernelGGL((k_cg_iter<T, DIM, P>), dim3(nb), dim3(L::NT), 0, s, cg, nv, vs, cf, g, tab, it, id, nb);
  return hipGetLastError();
}

template <typename T>
static hipError_t cg_iter_t(const CGStateT<T>& cg, int nv, const CoefT<T>& cf, const Geo& g, const T* tab, int it,
                            int id, hipStream_t s) {
  if (g.dim == 2) { SISDC_DISPATCH_P(g.P, return (cg_iter_dim_p<T, 2, PP>(cg, nv, cf, g, tab, it, id, s))); }
  if (g.dim == 3) { SISDC_DISPATCH_P(g.P, return (cg_iter_dim_p<T, 3, PP>(cg, nv, cf, g, tab, it, id, s))); }
  return hipErrorInvalidValue;
}

// Isotropic path: D = nu I constant on the level; hexahedra with P in
// {1, 3, 7} ((P+1)^2 lanes tile a wave) and quadrilaterals of any degree.
template <typename T>
static bool iso_path_t(const Geo& g, const CoefT<T>& cf) {
  const bool shape = (g.dim == 3 && (g.P == 1 || g.P == 3 || g.P == 7)) || (g.dim == 2 && g.P >= 1 && g.P <= 8);
  return shape && iso_coef(cf);
}

#define SISDC_DISPATCH_ISO(P_, BODY)                 \
  switch (P_) {                                      \
    case 1: { constexpr int PP = 1; BODY; } break;  \
    case 3: { constexpr int PP = 3; BODY; } break;  \
    case 7: { constexpr int PP = 7; BODY; } break;  \
    default: return hipErrorInvalidValue;            \
  }

// dispatch over (dim, P) of the isotropic path; BODY uses DD and PP
#define SISDC_DISPATCH_ISO_DIM(G_, BODY)                                                  \
  do {                                                                                    \
    if ((G_).dim == 3) { constexpr int DD = 3; SISDC_DISPATCH_ISO((G_).P, BODY); }        \
    if ((G_).dim == 2) { constexpr int DD = 2; SISDC_DISPATCH_P((G_).P, BODY); }          \
    return hipErrorInvalidValue;                                                          \
  } while (0)

// The Helmholtz diagonal of the first element of component 0 of an
// isotropic level (every element and component has the same one).
template <typename T>
static hipError_t iso_diag_first(T* diag, const CoefT<T>& cf, T dtm, T ctau, const Geo& g, const T* tab,
                                 hipStream_t s) {
  SISDC_DISPATCH_ISO_DIM(g, return (diag_dim_p<T, DD, PP>(diag, 1, cf, dtm, ctau, g, tab, s, true)));
}

// grid of the isotropic CG kernels: the same partial count as the matvec
template <int DIM, int P>
static int iso_grid(const Geo& g) {
  return std::min(elem_tiles<DIM, P>(g), kElemCap);
}

// Grid of the isotropic matvec: the workgroups that are resident at once
// (so that each XCD's interleaved window of pairs is the one in flight),
// at most kElemCap (partial sums) and at most one per lane group needed.
// The brick form of the hexahedral P = 7 matvec needs an even number of
// elements along every axis.
template <int DIM, int P>
static bool iso_brick(const Geo& g) {
  return DIM == 3 && P == 7 && g.ne[0] % 2 == 0 && g.ne[1] % 2 == 0 && g.ne[2] % 2 == 0 && g.wl % 2 == 0;
}

template <typename T, int DIM, int P>
static int iso_apply_grid(const Geo& g, int nv) {
  using K = IsoKernel<T, DIM, P>;
  if constexpr (DIM == 3 && P == 7) {
    if (iso_brick<DIM, P>(g)) {
      static const int resident_b = [] {
        int dev = 0, ncu = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_sipg_apply_iso3_brick<T, P>,
                                                         ISOB<P>::NT, 0) != hipSuccess)
          return kElemCap;
        return std::max(1, per_cu * ncu);
      }();
      const long tasks = (long)nv * (g.E / 8);
      return (int)std::max<long>(1, std::min<long>({(long)resident_b, (long)kElemCap, tasks}));
    }
  }
  static const int resident = [] {
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, K::fn(), K::NT, 0) != hipSuccess)
      return kElemCap;
    return std::max(1, per_cu * ncu);
  }();
  const long groups = ((long)nv * g.E + K::GPB - 1) / K::GPB;
  return (int)std::max<long>(1, std::min<long>({(long)resident, (long)kElemCap, groups}));
}

template <typename T, int DIM, int P>
static hipError_t apply_iso_p(const T* x, const T* isc, T* out, int nv, const CoefT<T>& cf, T alpha, T beta,
                              T ctau, const Geo& g, const T* tab, T* part, const int* done_gen, int id,
                              hipStream_t s) {
  const long vs = (long)g.E * EL<DIM, P>::NP;
  const int nb = iso_apply_grid<T, DIM, P>(g, nv);
  if constexpr (DIM == 3 && P == 7) {
    if (iso_brick<DIM, P>(g)) {
      hipLaunchKernelGGL((k_sipg_apply_iso3_brick<T, P>), dim3(nb), dim3(ISOB<P>::NT), 0, s, x, isc, out, nv, vs,
                         cf.nu, alpha, beta, ctau, g, tab, part, done_gen, id);
      return hipGetLastError();
    }
  }
  if constexpr (DIM == 3)
    hipLaunchKernelGGL((k_sipg_apply_iso3<T, P>), dim3(nb), dim3(ISO<P>::NT), 0, s, x, isc, out, nv, vs, cf.nu,
                       alpha, beta, ctau, g, tab, part, done_gen, id);
  else
    hipLaunchKernelGGL((k_sipg_apply_iso2<T, P>), dim3(nb), dim3(ISO2<P>::NT), 0, s, x, isc, out, nv, vs, cf.nu,
                       alpha, beta, ctau, g, tab, part, done_gen, id, (const T*)nullptr);
  return hipGetLastError();
}

template <typename T, int DIM, int P>
static hipError_t cg_start_iso_p(const CGStateT<T>& cg, const T* idg, int nv, const Geo& g, const LinComb* bl,
                                 const double* mw, hipStream_t s) {
  constexpr int NP = EL<DIM, P>::NP;
  if (!cg.b && (!bl || !mw)) return hipErrorInvalidValue;
  LinComb l{};
  if (!cg.b) l = *bl;
  hipLaunchKernelGGL((k_cg_start_iso<T, NP>), dim3(iso_grid<DIM, P>(g)), dim3(1024), 0, s, cg, idg,
                     (long)nv * g.E * NP, l, mw);
  return hipGetLastError();
}

template <typename T, int DIM, int P>
static hipError_t cg_iter_iso_p(const CGStateT<T>& cg, const T* idg, int nv, const Geo& g, int it, int id,
                                hipStream_t s) {
  constexpr int NP = EL<DIM, P>::NP;
  const int nb = iso_grid<DIM, P>(g);
  const long n = (long)nv * g.E * NP;
  const int nd = iso_apply_grid<T, DIM, P>(g, nv);
  if (cg.zs && cg.cons)
    hipLaunchKernelGGL((k_cg_iter_iso<T, NP, true, true>), dim3(nb), dim3(1024), 0, s, cg, idg, n, it, id, nb, nd);
  else if (cg.zs)
    hipLaunchKernelGGL((k_cg_iter_iso<T, NP, true, false>), dim3(nb), dim3(1024), 0, s, cg, idg, n, it, id, nb, nd);
  else if (cg.cons)
    hipLaunchKernelGGL((k_cg_iter_iso<T, NP, false, true>), dim3(nb), dim3(1024), 0, s, cg, idg, n, it, id, nb, nd);
  else
    hipLaunchKernelGGL((k_cg_iter_iso<T, NP, false, false>), dim3(nb), dim3(1024), 0, s, cg, idg, n, it, id, nb, nd);
  return hipGetLastError();
}

template <int DIM, int P>
static hipError_t fds_dim_p(const double* r, double* z, int nv, const Geo& g, const double* fds, double dtk,
                            double* part_rz, double* part_rr, const int* done_gen, int id, hipStream_t s) {
  using L = EL<DIM, P>;
  const int tiles = elem_tiles<DIM, P>(g);
  // with partials: the grid of the streaming CG kernels, whose partial counts they replace
  const int nb = part_rz ? iso_grid<DIM, P>(g) : std::max(1, std::min(nv * tiles, 4096));
  hipLaunchKernelGGL((k_fds_apply<double, DIM, P>), dim3(nb), dim3(L::NT), 0, s, r, z, nv, g, fds, dtk, part_rz,
                     part_rr, done_gen, id);
  return hipGetLastError();
}

hipError_t launch_fds(const double* r, double* z, int nv, const Geo& g, const double* fds, double dtk,
                      double* part_rz, double* part_rr, const int* done_gen, int id, hipStream_t s) {
  SISDC_DISPATCH(g, fds_dim_p, r, z, nv, g, fds, dtk, part_rz, part_rr, done_gen, id, s);
}

// Grid of the streaming isotropic CG's start and update kernels on a level
// (the count of their block partials); 0 where that path does not apply.
int iso_cg_grid(const Geo& g) {
  if (g.dim == 3) {
    switch (g.P) {
      case 1: return iso_grid<3, 1>(g);
      case 3: return iso_grid<3, 3>(g);
      case 7: return iso_grid<3, 7>(g);
      default: return 0;
    }
  }
  if (g.dim == 2) {
    switch (g.P) {
      case 1: return iso_grid<2, 1>(g);
      case 2: return iso_grid<2, 2>(g);
      case 3: return iso_grid<2, 3>(g);
      case 4: return iso_grid<2, 4>(g);
      case 5: return iso_grid<2, 5>(g);
      case 6: return iso_grid<2, 6>(g);
      case 7: return iso_grid<2, 7>(g);
      case 8: return iso_grid<2, 8>(g);
      default: return 0;
    }
  }
  return 0;
}

#define SISDC_PRECISION_LAUNCHERS(T)                                                                            \
  hipError_t launch_sipg_trace(const T* x, int nv, const CoefT<T>& cf, T* trace, const Geo& g, const T* tab,     \
                               hipStream_t s) {                                                                 \
    return sipg_trace_t<T>(x, nv, cf, trace, g, tab, s);                                                        \
  }                                                                                                             \
  hipError_t launch_sipg_apply(const T* x, T* out, int nv, const CoefT<T>& cf, const T* trace, T alpha, T beta, \
                               T ctau, const Geo& g, const T* tab, const T* dotv, T* part, const int* done_gen, \
                               int id, hipStream_t s) {                                                         \
    return sipg_apply_t<T>(x, out, nv, cf, trace, alpha, beta, ctau, g, tab, dotv, part, done_gen, id, s);      \
  }                                                                                                             \
  hipError_t launch_sipg(const T* x, T* out, int nv, const CoefT<T>& cf, T* trace, T alpha, T beta, T ctau,     \
                         const Geo& g, const T* tab, hipStream_t s) {                                           \
    if (!iso_path_t<T>(g, cf)) { /* the isotropic kernel needs no trace pass */                                 \
      hipError_t e = sipg_trace_t<T>(x, nv, cf, trace, g, tab, s);                                              \
      if (e != hipSuccess) return e;                                                                            \
    }                                                                                                           \
    return sipg_apply_t<T>(x, out, nv, cf, trace, alpha, beta, ctau, g, tab, nullptr, nullptr, nullptr, 0, s);  \
  }                                                                                                             \
  hipError_t launch_helm_diag(T* diag, int nv, const CoefT<T>& cf, T dtm, T ctau, const Geo& g, const T* tab,    \
                              hipStream_t s) {                                                                  \
    return helm_diag_t<T>(diag, nv, cf, dtm, ctau, g, tab, s);                                                  \
  }                                                                                                             \
  hipError_t launch_cg_start(const CGStateT<T>& cg, int nv, const CoefT<T>& cf, const Geo& g, const T* tab,     \
                             hipStream_t s) {                                                                   \
    return cg_start_t<T>(cg, nv, cf, g, tab, s);                                                                \
  }                                                                                                             \
  hipError_t launch_cg_iter(const CGStateT<T>& cg, int nv, const CoefT<T>& cf, const Geo& g, const T* tab,      \
                            int it, int id, hipStream_t s) {                                                    \
    return cg_iter_t<T>(cg, nv, cf, g, tab, it, id, s);                                                         \
  }                                                                                                             \
  bool sipg_iso_path(const Geo& g, const CoefT<T>& cf) { return iso_path_t<T>(g, cf); }                         \
  hipError_t launch_iso_inv_diag(T* diag, T* idg, const CoefT<T>& cf, T dtm, T ctau, const Geo& g, const T* tab, \
                                 hipStream_t s) {                                                               \
    if (!iso_path_t<T>(g, cf)) return hipErrorInvalidValue;                                                     \
    const hipError_t e = iso_diag_first<T>(diag, cf, dtm, ctau, g, tab, s);                                     \
    if (e != hipSuccess) return e;                                                                              \
    const int np = g.dim == 3 ? (g.P + 1) * (g.P + 1) * (g.P + 1) : (g.P + 1) * (g.P + 1);                     \
    hipLaunchKernelGGL((k_inv_table<T>), dim3((np + 255) / 256), dim3(256), 0, s, diag, idg, np);               \
    return hipGetLastError();                                                                                   \
  }                                                                                                             \
  hipError_t launch_sipg_apply_iso(const T* x, const T* isc, T* out, int nv, const CoefT<T>& cf, T alpha,       \
                                   T beta, T ctau, const Geo& g, const T* tab, T* part, const int* done_gen,    \
                                   int id, hipStream_t s) {                                                     \
    if (!iso_path_t<T>(g, cf)) return hipErrorInvalidValue;                                                     \
    SISDC_DISPATCH_ISO_DIM(g, return (apply_iso_p<T, DD, PP>(x, isc, out, nv, cf, alpha, beta, ctau, g, tab,    \
                                                             part, done_gen, id, s)));                          \
  }                                                                                                             \
  hipError_t launch_cg_start_iso(const CGStateT<T>& cg, const T* idg, int nv, const Geo& g, const LinComb* bl,   \
                                 const double* mw, hipStream_t s) {                                             \
    SISDC_DISPATCH_ISO_DIM(g, return (cg_start_iso_p<T, DD, PP>(cg, idg, nv, g, bl, mw, s)));                   \
  }                                                                                                             \
  hipError_t launch_cg_iter_iso(const CGStateT<T>& cg, const T* idg, int nv, const Geo& g, int it, int id,      \
                                hipStream_t s) {                                                                \
    SISDC_DISPATCH_ISO_DIM(g, return (cg_iter_iso_p<T, DD, PP>(cg, idg, nv, g, it, id, s)));                    \
  }                                                                                                             \
  hipError_t launch_cg_fix_iso(const CGStateT<T>& cg, long n, int id, hipStream_t s) {                          \
    hipLaunchKernelGGL((k_cg_fix_iso<T>), dim3(blocks_for(n, 256, 2048)), dim3(256), 0, s, cg, n, id);          \
    return hipGetLastError();                                                                                   \
  }

SISDC_PRECISION_LAUNCHERS(double)
SISDC_PRECISION_LAUNCHERS(float)

template <int DIM, int P>
static hipError_t visc_dim_p(const double* u, const double* add, double* out, double* trace, const Geo& g,
                             const EqP& q, const double* tab, hipStream_t s) {
  using L = EL<DIM, P>;
  const long vs = (long)g.E * L::NP;
  hipLaunchKernelGGL((k_visc_trace<DIM, P>), dim3(elem_tiles<DIM, P>(g)), dim3(L::NTF), 0, s, u, trace, g, q, tab, vs);
  hipLaunchKernelGGL((k_visc_apply<DIM, P>), dim3(elem_tiles<DIM, P>(g)), dim3(L::NTF), 0, s, u, out, trace, g, q, tab,
                     vs, add);
  return hipGetLastError();
}

hipError_t launch_visc(const double* u, const double* add, double* out, double* trace, const Geo& g, const EqP& q,
                       const double* tab, hipStream_t s) {
  if (add == out) add = nullptr;  // in place: out += V(u)
  SISDC_DISPATCH(g, visc_dim_p, u, add, out, trace, g, q, tab, s);
}

hipError_t launch_lincomb(double* out, const LinComb& lc, long n, const double* mw, int np, hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, out, lc, n, mw, np);
  return hipGetLastError();
}

hipError_t launch_colloc_residual(const CollocResid& c, long n, const double* mw, int np, hipStream_t s) {
  if (c.M < 1 || c.M > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_colloc_residual, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, c, n, mw, np);
  return hipGetLastError();
}

hipError_t launch_space_time_transfer(const TransferMulti& t, int nv, int dim, int n1i, int n1o, int E,
                                      const double* A, hipStream_t s) {
  if (t.nin < 1 || t.nin > kTransferIn || t.nout < 1 || t.nout > kTransferOut || n1i > kMaxP + 1 ||
      n1o > kMaxP + 1 || (dim != 2 && dim != 3))
    return hipErrorInvalidValue;
  const int npi = dim == 2 ? n1i * n1i : n1i * n1i * n1i;
  const int n1m = std::max(n1i, n1o);
  const int nbuf = dim == 2 ? n1m * n1m : n1m * n1m * n1m;
  const size_t lds = sizeof(double) * ((size_t)n1i * n1o + (size_t)t.nout * npi + 2 * (size_t)nbuf);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_space_time_transfer, dim3((unsigned)((long)nv * E)), dim3(256), lds, s, t, dim, n1i, n1o, A);
  return hipGetLastError();
}

hipError_t launch_space_transfer(const double* in, double* out, int nv, int dim, int n1i, int n1o, int E,
                                 const double* A, hipStream_t s) {
  hipLaunchKernelGGL(k_space_transfer, dim3((unsigned)((long)nv * E)), dim3(256), 0, s, in, out, dim, n1i, n1o,
                     E, A);
  return hipGetLastError();
}

template <int P>
static hipError_t iso2_add_p(const double* x, const double* add, double* out, int nv, const CoefT<double>& cf,
                             double alpha, double beta, double ctau, const Geo& g, const double* tab, hipStream_t s) {
  using K = IsoKernel<double, 2, P>;
  const long vs = (long)g.E * (P + 1) * (P + 1);
  const long groups = ((long)nv * g.E + K::GPB - 1) / K::GPB;
  const int nbi = (int)std::min<long>(std::max<long>(groups, 1), 8192);
  hipLaunchKernelGGL((k_sipg_apply_iso2<double, P>), dim3(nbi), dim3(K::NT), 0, s, x, (const double*)nullptr, out,
                     nv, vs, cf.nu, alpha, beta, ctau, g, tab, (double*)nullptr, (const int*)nullptr, 0, add);
  return hipGetLastError();
}

hipError_t launch_sipg_iso2_add(const double* x, const double* add, double* out, int nv, const CoefT<double>& cf,
                                double alpha, double beta, double ctau, const Geo& g, const double* tab,
                                hipStream_t s) {
  if (g.dim != 2 || !iso_path_t<double>(g, cf)) return hipErrorInvalidValue;
  SISDC_DISPATCH_P(g.P, return (iso2_add_p<PP>(x, add, out, nv, cf, alpha, beta, ctau, g, tab, s)));
  return hipErrorInvalidValue;
}

hipError_t launch_lincomb_multi(double* out, const LinCombMulti& lc, long n, hipStream_t s) {
  if (lc.nin < 1 || lc.nin > 8 || lc.nout < 1 || lc.nout > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lincomb_multi, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, out, lc, n);
  return hipGetLastError();
}

hipError_t launch_space_transfer_h(const double* in, double* out, int nv, int dim, int n1f, int n1c, const int* nc,
                                   const double* A, int mode, hipStream_t s) {
  const int S = 2 * n1f;
  const long grid = dim == 2 ? (long)S * S : (long)S * S * S;
  if (grid > kHGrid || n1f > kMaxP + 1 || n1c > kMaxP + 1 || n1c > S || (dim != 2 && dim != 3))
    return hipErrorInvalidValue;
  const int ncz = dim == 3 ? nc[2] : 1;
  const long blocks = (long)nv * nc[0] * nc[1] * ncz;
  hipLaunchKernelGGL(k_space_transfer_h, dim3((unsigned)blocks), dim3(256), 0, s, in, out, dim, n1f, n1c, nc[0],
                     nc[1], ncz, A, mode);
  return hipGetLastError();
}

hipError_t launch_copy(const double* in, double* out, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_cast_f(const double* in, float* out, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_resid_cast(const double* b, const double* Ax, float* r32, long n, double* part, double* tot,
                             hipStream_t s) {
  const int nb = blocks_for(n, 256, kElemCap);
  hipLaunchKernelGGL(k_resid_cast, dim3(nb), dim3(256), 0, s, b, Ax, r32, n, part);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, part, nb, tot);
  return hipGetLastError();
}

hipError_t launch_dot2(const double* a, const double* b, const double* c, long n, double* part, double* tot,
                       hipStream_t s) {
  const int nb = blocks_for(n, 256, kElemCap);
  hipLaunchKernelGGL(k_dot2, dim3(nb), dim3(256), 0, s, a, b, c, n, part);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, part, nb, tot);
  return hipGetLastError();
}

hipError_t launch_conserve(const double* b, const LinComb* lc, double* x, int nv, long vs, const double* mw, int np,
                           double mass_total, double* part, int part_cap, hipStream_t s) {
  if (nv < 1 || part_cap < 2 * nv || !(mass_total > 0.0) || (!b && !lc)) return hipErrorInvalidValue;
  const int nb = std::max(1, std::min(blocks_for(vs, 256, kElemCap), part_cap / (2 * nv)));
  LinComb l{};
  if (!b) l = *lc;
  hipLaunchKernelGGL(k_conserve_sums, dim3(nb, nv), dim3(256), 0, s, b, l, (const double*)x, vs, mw, np, part);
  hipLaunchKernelGGL(k_conserve_apply, dim3(blocks_for(vs, 256, 1024), nv), dim3(256), 0, s, x, vs,
                     (const double*)part, nb, mass_total);
  return hipGetLastError();
}

hipError_t launch_add_f2d(double* x, const float* e, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f2d, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, x, e, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- artificial viscosity
// Persson-Peraire viscosity of one element per workgroup (Sec. 6 supplements
// the diffusion matrix with it): the coefficients of component 0 in the
// orthonormal Legendre tensor basis (the discrete transform A, applied along
// each axis in LDS), the share S of their energy in the modes with some index
// equal to P, and the largest wave speed over the element's nodes and the
// axes; then eps_e = ceps lam_e sw(log10 S) with the sine switch of
// half-width kappa around s0 (eps_e = 0 for S = 0).  The sums run in a fixed
// order (per thread, then the waves in turn), so eps is deterministic.
template <int DIM, int P>
struct AVS {
  static constexpr int N1 = P + 1, NP = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
  static constexpr int NT = ((NP + 63) / 64) * 64 > 512 ? 512 : ((NP + 63) / 64) * 64;
  static constexpr int NW = NT / 64;
};

template <int DIM, int P, int NV>
__global__ void __launch_bounds__((AVS<DIM, P>::NT))
k_av_sensor(const double* __restrict__ u, long vs, EqP q, int E, const double* __restrict__ A, double s0, double kappa,
            double ceps, double* __restrict__ eps) {
  using K = AVS<DIM, P>;
  constexpr int N1 = K::N1, NP = K::NP, NT = K::NT, NW = K::NW;
  __shared__ double sa[NP], sb[NP], sA[N1 * N1];
  __shared__ double red[3][NW];
  const int e = blockIdx.x, t = threadIdx.x;
  if (e >= E) return;
  for (int k = t; k < N1 * N1; k += NT) sA[k] = A[k];
  double lam = 0.0;
  for (int n = t; n < NP; n += NT) {
    const long i = (long)e * NP + n;
    double uv[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) uv[c] = u[c * vs + i];
    sa[n] = uv[0];
    for (int d = 0; d < DIM; ++d) lam = fmax(lam, wave_speed<NV>(q, d, uv));
  }
  __syncthreads();
  // transform along x (fastest), then y (then z); each pass reads one buffer
  // and writes the other
  double* src = sa;
  double* dst = sb;
#pragma unroll
  for (int ax = 0; ax < DIM; ++ax) {
    const int st = ax == 0 ? 1 : (ax == 1 ? N1 : N1 * N1);
    for (int n = t; n < NP; n += NT) {
      const int k = (n / st) % N1;
      const int base = n - k * st;
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < N1; ++i) acc += sA[k * N1 + i] * src[base + i * st];
      dst[n] = acc;
    }
    __syncthreads();
    double* tmp = src;
    src = dst;
    dst = tmp;
  }
  double tot = 0.0, top = 0.0;
  for (int n = t; n < NP; n += NT) {
    const double c = src[n];
    const int k0 = n % N1, k1 = (n / N1) % N1, k2 = DIM == 3 ? n / (N1 * N1) : 0;
    tot += c * c;
    if (k0 == P || k1 == P || (DIM == 3 && k2 == P)) top += c * c;
  }
  for (int off = 32; off > 0; off >>= 1) {
    tot += __shfl_down(tot, off, 64);
    top += __shfl_down(top, off, 64);
    lam = fmax(lam, __shfl_down(lam, off, 64));
  }
  if ((t & 63) == 0) {
    red[0][t >> 6] = tot;
    red[1][t >> 6] = top;
    red[2][t >> 6] = lam;
  }
  __syncthreads();
  if (t != 0) return;
  double T0 = 0.0, T1 = 0.0, L = 0.0;
  for (int w = 0; w < NW; ++w) {
    T0 += red[0][w];
    T1 += red[1][w];
    L = fmax(L, red[2][w]);
  }
  double sw = 0.0;
  if (T0 > 0.0 && T1 > 0.0) {
    const double sl = log10(T1 / T0);
    if (sl > s0 + kappa)
      sw = 1.0;
    else if (sl >= s0 - kappa)
      sw = 0.5 * (1.0 + sin(M_PI * (sl - s0) / (2.0 * kappa)));
  }
  eps[e] = ceps * L * sw;
}

template <int DIM, int P>
static hipError_t av_dim_p(const double* u, int nv, const Geo& g, const EqP& q, const double* A, double s0,
                           double kappa, double ceps, double* eps, hipStream_t s) {
  using K = AVS<DIM, P>;
  const long vs = (long)g.E * K::NP;
  if (nv == 1)
    hipLaunchKernelGGL((k_av_sensor<DIM, P, 1>), dim3(g.E), dim3(K::NT), 0, s, u, vs, q, g.E, A, s0, kappa, ceps, eps);
  else if (nv == DIM + 2)
    hipLaunchKernelGGL((k_av_sensor<DIM, P, DIM + 2>), dim3(g.E), dim3(K::NT), 0, s, u, vs, q, g.E, A, s0, kappa,
                       ceps, eps);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_av_sensor(const double* u, int nv, const Geo& g, const EqP& q, const double* A, double kappa,
                            double c_s, double* eps, hipStream_t s) {
  if (g.E < 1 || !(kappa > 0.0)) return hipErrorInvalidValue;
  const double s0 = -4.0 * std::log10((double)g.P);
  double hmin = g.h[0];
  for (int d = 1; d < g.dim; ++d) hmin = std::min(hmin, g.h[d]);
  const double ceps = c_s * hmin / g.P;
  if (g.dim == 2) { SISDC_DISPATCH_P(g.P, return (av_dim_p<2, PP>(u, nv, g, q, A, s0, kappa, ceps, eps, s))); }
  if (g.dim == 3) { SISDC_DISPATCH_P(g.P, return (av_dim_p<3, PP>(u, nv, g, q, A, s0, kappa, ceps, eps, s))); }
  return hipErrorInvalidValue;
}

hipError_t launch_euler_lam(const double* u, long vs, const EqP& q, int dim, double* part, double* result,
                            hipStream_t s) {
  const int nb = blocks_for(vs, 256, kElemCap);
  if (dim == 2)
    hipLaunchKernelGGL(k_euler_lam<2>, dim3(nb), dim3(256), 0, s, u, vs, q, part);
  else
    hipLaunchKernelGGL(k_euler_lam<3>, dim3(nb), dim3(256), 0, s, u, vs, q, part);
  hipLaunchKernelGGL(k_maxmin_partials, dim3(1), dim3(256), 0, s, part, nb, result);
  return hipGetLastError();
}

}  // namespace sisdc
