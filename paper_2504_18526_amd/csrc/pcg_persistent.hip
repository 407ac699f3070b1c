// Persistent Jacobi-PCG for levels whose elements fit on the GPU at once:
// one launch per Helmholtz solve (M + dt_m K_D) x = b, with a grid no larger
// than the number of workgroups the device holds at once (from the occupancy
// query), so every workgroup is resident while the others wait for it.
//
// Every workgroup owns one tile of EPB elements for the whole solve; a
// thread owns one node and keeps the CG vectors and the Jacobi diagonal in
// registers.  The iteration is the pipelined form of preconditioned CG
// (Ghysels & Vanroose): the global reduction of (r,u), (w,u), (r,r) travels
// with the face data of m = diag^-1 w, so each iteration needs ONE grid
// barrier.  The only data that leave a workgroup are the face values and
// face traces (D grad m) of its elements and three partial sums; they are
// written with device-scope stores and read with device-scope loads (both go
// through to the point of coherence; no L2 write-back is needed), each
// 64-bit word carrying 32 bits of a value and the 32-bit tag of its barrier,
// so a reader validates what it loads and no flag or store ordering is
// needed.  The volume part of the next matvec and the loads of the
// neighbours' face words run while a barrier waits.  The right-hand side is
// given, or formed at every node from up to eight vectors.  When the
// recurred residual meets the tolerance the true residual b - A x is
// computed; if it misses the tolerance (the recurrences drifted), r, u and w
// are replaced by their true values and the iteration continues.  The
// recurrences of the pipelined form lose accuracy near 1e-12, so the host
// uses this solver for tolerances >= 1e-11 only.
//
// The grid barrier is an all-gather of per-workgroup records (no atomics,
// one writer per word) with bounded spins: a barrier that does
// not complete within spin_limit polls sets the abort word and every
// workgroup leaves, so the kernel always ends.
//
// Convergence decisions are made by every workgroup from the same partial
// sums summed in the same order, so all workgroups take the same branch.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"
#include "xcd.hpp"

namespace sisdc {

namespace {

// Tile of one workgroup: EPB whole elements, one node per thread, up to 512
// threads; elements of at most 32 nodes take 256-thread tiles, since the grid
// barrier's latency, not the workgroup count, bounds those small levels.
template <int DIM, int P>
struct PT {
  static constexpr int N1 = P + 1;
  static constexpr int NP = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
  static constexpr int NF = DIM == 2 ? N1 : N1 * N1;
  static constexpr int EPB = NP >= 512 ? 1 : (NP <= 32 ? 256 : 512) / NP;
  static constexpr int NT = ((EPB * NP + 63) / 64) * 64;
  static constexpr int stride(int d) { return d == 0 ? 1 : (d == 1 ? N1 : N1 * N1); }
};



__device__ __forceinline__ void st_dev64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_dev64(const unsigned long long* p) {
  return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A double published as two words, 32 bits of it and the tag in each.
__device__ __forceinline__ void st_tagged(unsigned long long* p, double v, unsigned long long tag_hi) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  st_dev64(p, tag_hi | (b & 0xffffffffull));
  st_dev64(p + 1, tag_hi | (b >> 32));
}
__device__ __forceinline__ double untag(unsigned long long lo, unsigned long long hi) {
  return __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
}

// All-gather grid barrier with reduction.  Each workgroup stores its K block
// sums in its own record (word j of workgroup b at rec[j * cap + b], so the
// readers' loads of one word of consecutive records coalesce), every 64-bit
// word carrying 32 bits of a sum and
// the barrier's tag (a number no record holds when the launch starts) in its
// upper half, so a word is valid exactly when its tag matches: a reader
// needs no separate flag and no second load, and the writer no wait between
// the sums and a flag.  Every workgroup waits until all records carry the
// tag and sums them in workgroup order (thread t takes records t,
// t + blockDim, ...; the same shuffle and LDS order everywhere), so all
// workgroups obtain the same bits.  No atomics: every word has one writer.
// The face data carry tags of their own, so the record is not ordered after
// them: a reader waits for a face word's tag where it uses it.  Bounded
// spins: returns false (and sets the abort word) when a wait exceeds
// spin_limit polls.
// `overlap` is work of the whole workgroup that needs no other workgroup's
// data: it runs after the record is stored, while the other records arrive.
template <int K, typename F>
__device__ bool sync_reduce(const double (&v)[K], double (&tot)[K], unsigned long long* rec, long cap,
                            unsigned* abort_w, unsigned tag, long spin_limit, int* s_ok, F&& overlap) {
  static_assert(K >= 1 && K <= 8, "a record holds up to 8 values");
  // LDS sums by barrier parity (tag & 1): a barrier rewrites the ones of the
  // barrier two before it, which every thread has left by the first
  // __syncthreads of the barrier in between, so none is needed at the end
  __shared__ double sred2[2][K][16];
  __shared__ double stot2[2][K][16];
  double (&sred)[K][16] = sred2[tag & 1u];
  double (&stot)[K][16] = stot2[tag & 1u];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int k = 0; k < K; ++k) {
    const double x = wave_sum63(v[k]);
    if (lane == 63) sred[k][wid] = x;
  }
  if (threadIdx.x == 0) *s_ok = 1;
  __syncthreads();
  const unsigned long long hi = (unsigned long long)tag << 32;
  if (threadIdx.x == 0) {
    unsigned long long* my = rec + blockIdx.x;
    for (int k = 0; k < K; ++k) {
      double sb = 0.0;
      for (int w = 0; w < nw; ++w) sb += sred[k][w];
      const unsigned long long bits = (unsigned long long)__double_as_longlong(sb);
      st_dev64(&my[(2 * k) * cap], hi | (bits & 0xffffffffull));
      st_dev64(&my[(2 * k + 1) * cap], hi | (bits >> 32));
    }
  }
  overlap();
  double acc[K];
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  int ok = 1;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
    const unsigned long long* rb = rec + b;
    unsigned long long wv[2 * K];
    long spins = 0;
    while (true) {
      // poll one word; once it carries the tag, read the others (they were
      // stored together, so they are normally there as well)
      wv[2 * K - 1] = ld_dev64(&rb[(2 * K - 1) * cap]);
      if ((wv[2 * K - 1] >> 32) == (unsigned long long)tag) {
        for (int j = 0; j < 2 * K - 1; ++j) wv[j] = ld_dev64(&rb[j * cap]);
        bool ready = true;
        for (int j = 0; j < 2 * K - 1; ++j) ready = ready && (wv[j] >> 32) == (unsigned long long)tag;
        if (ready) break;
      }
      // the abort word is read every 64th poll only: a load of it in every
      // poll would double the time a poll takes
      if ((++spins & 63) == 0 &&
          (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spins > spin_limit)) {
        __hip_atomic_store(abort_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!ok) break;
    for (int k = 0; k < K; ++k)
      acc[k] += __longlong_as_double((long long)((wv[2 * k + 1] << 32) | (wv[2 * k] & 0xffffffffull)));
  }
  if (!ok) *s_ok = 0;  // benign race: every writer stores 0
  for (int k = 0; k < K; ++k) {
    const double x = wave_sum63(acc[k]);
    if (lane == 63) stot[k][wid] = x;
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    double sb = 0.0;
    for (int w = 0; w < nw; ++w) sb += stot[k][w];
    tot[k] = sb;
  }
  return *s_ok != 0;
}

// periodic neighbour; along the last axis within the instance's g.wl elements
__device__ __forceinline__ int nbr(const Geo& g, int e, int d, int s) {
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

template <int DIM, int N1>
__device__ __forceinline__ int fidx(int d, const int (&i)[3]) {
  if (DIM == 2) return i[1 - d];
  return d == 0 ? i[1] + N1 * i[2] : (d == 1 ? i[0] + N1 * i[2] : i[0] + N1 * i[1]);
}

}  // namespace

template <int DIM, int P, int NV>
__global__ void __launch_bounds__((PT<DIM, P>::NT))
k_pcg_persistent(PCGArgs a, CoefP cf, Geo g, const double* __restrict__ tab) {
  using L = PT<DIM, P>;
  constexpr int N1 = L::N1, NP = L::NP, NF = L::NF, EPB = L::EPB;
  __shared__ double sD[N1 * N1], sw[N1];
  __shared__ double sx[NV * EPB * NP];
  __shared__ double sQ[EPB * DIM * NP];
  __shared__ double sc[EPB * NP];
  __shared__ int s_ok[2];  // barrier outcome, by barrier parity (see sync_reduce)
  const int t = threadIdx.x, le = t / NP, n = t - le * NP;
  const int e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool act = (le < EPB) && (e < g.E);
  const long vs = (long)g.E * NP;
  const long own = (long)e * NP + n;
  for (int k = t; k < N1 * N1; k += blockDim.x) sD[k] = tab[k];
  for (int k = t; k < N1; k += blockDim.x) sw[k] = tab[N1 * N1 + k];
  int ii[3];
  ii[0] = n % N1;
  ii[1] = (n / N1) % N1;
  ii[2] = DIM == 3 ? n / (N1 * N1) : 0;
  const double cw = act ? (cf.ub ? cf.c * cf.ub[own] * cf.ub[own] : cf.c) : 0.0;
  if (act) sc[le * NP + n] = cw;
  __syncthreads();
  unsigned gen = 0u;  // barriers passed in this launch
  double wn = 1.0;
  for (int d = 0; d < DIM; ++d) wn *= sw[ii[d]];
  const double jw = g.J * wn;
  const double pen = a.ctau * (double)(N1 * N1);

  // neighbour coefficient D_dd at the face nodes (read-only during the solve)
  double dnb[DIM][2];
  for (int d = 0; d < DIM; ++d)
    for (int side = 0; side < 2; ++side) {
      dnb[d][side] = 0.0;
      if (act && ii[d] == (side ? P : 0)) {
        const int nb = nbr(g, e, d, side ? 1 : -1);
        const int nn = n + ((side ? 0 : P) - ii[d]) * L::stride(d);
        const long nbi = (long)nb * NP + nn;
        const double cwn = cf.ub ? cf.c * cf.ub[nbi] * cf.ub[nbi] : cf.c;
        dnb[d][side] = cwn * cf.v[d] * cf.v[d] + cf.nu;
      }
    }

  // Jacobi diagonal (same formula as the multi-kernel path)
  double dg = 1.0;
  if (act) {
    double kd = 0.0;
    for (int d = 0; d < DIM; ++d) {
      const int st = L::stride(d);
      double s = 0.0;
      for (int k = 0; k < N1; ++k) {
        const int nk = n + (k - ii[d]) * st;
        const double dd = sc[le * NP + nk] * cf.v[d] * cf.v[d] + cf.nu;
        const double wk = wn / sw[ii[d]] * sw[k];
        s += sD[k * N1 + ii[d]] * sD[k * N1 + ii[d]] * wk * dd;
      }
      kd += g.rh2[d] * g.rh2[d] * g.J * s;
    }
    for (int d = 0; d < DIM; ++d)
      for (int side = 0; side < 2; ++side) {
        if (ii[d] != (side ? P : 0)) continue;
        const double sgn = side ? 1.0 : -1.0;
        const double dow = cw * cf.v[d] * cf.v[d] + cf.nu;
        const double tau = pen * fmax(dow, dnb[d][side]) * 0.5 * g.rh2[d];
        const double jfwf = g.J * g.rh2[d] * wn / sw[ii[d]];
        kd += jfwf * (tau - sgn * g.rh2[d] * dow * sD[ii[d] * N1 + ii[d]]);
      }
    dg = jw + a.dtm * kd;
  }

  // Face data are double-buffered by barrier parity: a workgroup may publish
  // the next vector while a slower neighbour still reads the previous one.
  // Every face value is stored as two words tagged with the barrier that
  // follows the publish, so a reader can load it before that barrier has
  // passed (while the barrier waits) and keep it if both tags match.
  const long fsize = 2L * NV * g.E * DIM * 2 * NF;  // words per buffer
  long fofs = 0;                                   // buffer of the last publish
  unsigned ftag = 0;                               // its tag
  // publish: stage v in LDS, store its face values and face traces
  auto publish = [&](const double (&v)[NV]) {
    fofs = (long)(gen & 1u) * fsize;
    ftag = a.tag0 + gen;
    const unsigned long long tag_hi = (unsigned long long)ftag << 32;
    for (int c = 0; c < NV; ++c)
      if (act) sx[(c * EPB + le) * NP + n] = v[c];
    __syncthreads();
    if (!act) return;
    bool face = false;
    for (int d = 0; d < DIM; ++d) face = face || ii[d] == 0 || ii[d] == P;
    if (!face) return;
    for (int c = 0; c < NV; ++c) {
      const double* tile = &sx[(c * EPB + le) * NP];
      double gr[DIM];
      for (int d = 0; d < DIM; ++d) {
        const int st = L::stride(d);
        const double* row = &tile[n - ii[d] * st];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < N1; ++k) s += sD[ii[d] * N1 + k] * row[k * st];
        gr[d] = g.rh2[d] * s;
      }
      double vg = 0.0;
      for (int j = 0; j < DIM; ++j) vg += cf.v[j] * gr[j];
      for (int d = 0; d < DIM; ++d) {
        const bool lo = ii[d] == 0, hi = ii[d] == P;
        if (!lo && !hi) continue;
        const double qd = cw * cf.v[d] * vg + cf.nu * gr[d];
        const long base = 2 * ((((long)c * g.E + e) * DIM + d) * 2 * NF + fidx<DIM, N1>(d, ii) + (hi ? NF : 0));
        st_tagged(&a.ft[fofs + base], qd, tag_hi);
        st_tagged(&a.fz[fofs + base], v[c], tag_hi);
      }
    }
  };

  // the neighbours' face words this node needs (face value and trace, two
  // words each, per face of the node), loaded ahead by prefetch_faces()
  unsigned long long pf[NV][DIM][4];
  auto face_word = [&](int c, int d) -> long {
    const int side = ii[d] == P ? 1 : 0;
    const int nb = nbr(g, e, d, side ? 1 : -1);
    return fofs + 2 * ((((long)c * g.E + nb) * DIM + d) * 2 * NF + (side ? 0 : NF) + fidx<DIM, N1>(d, ii));
  };
  // (2-D only: in 3-D the words held across the barrier would not fit the
  // register budget; there face_vals loads them after the barrier)
  auto prefetch_faces = [&]() __attribute__((always_inline)) {
    if constexpr (DIM == 3) return;
    if (!act) return;
#pragma unroll
    for (int c = 0; c < NV; ++c)
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        if (ii[d] != 0 && ii[d] != P) continue;
        const long w = face_word(c, d);
        pf[c][d][0] = ld_dev64(&a.fz[w]);
        pf[c][d][1] = ld_dev64(&a.fz[w + 1]);
        pf[c][d][2] = ld_dev64(&a.ft[w]);
        pf[c][d][3] = ld_dev64(&a.ft[w + 1]);
      }
  };
  unsigned* abort_w = &a.bar[64];
  // after the barrier: the face value and trace of the neighbour across face
  // d, from the prefetched words, reloaded until they carry the tag of this
  // exchange (the neighbour has passed its publish, so they are on their way)
  auto face_vals = [&](int c, int d, double& xnb, double& qnb) __attribute__((always_inline)) {
    unsigned long long w0 = 0ull, w1 = 0ull, w2 = 0ull, w3 = 0ull;  // tag 0 is never published
    if constexpr (DIM == 2) {
      w0 = pf[c][d][0];
      w1 = pf[c][d][1];
      w2 = pf[c][d][2];
      w3 = pf[c][d][3];
    }
    const unsigned long long want = (unsigned long long)ftag;
    long spins = 0;
    while ((w0 >> 32) != want || (w1 >> 32) != want || (w2 >> 32) != want || (w3 >> 32) != want) {
      if (++spins > a.spin_limit) {
        __hip_atomic_store(abort_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      const long w = face_word(c, d);
      w0 = ld_dev64(&a.fz[w]);
      w1 = ld_dev64(&a.fz[w + 1]);
      w2 = ld_dev64(&a.ft[w]);
      w3 = ld_dev64(&a.ft[w + 1]);
    }
    xnb = untag(w0, w1);
    qnb = untag(w2, w3);
  };

  // out = M v + dt_m K_D v for v staged in LDS by publish(), in two parts:
  // apply_local takes every term that needs no neighbour data (mass term,
  // volume terms of both contractions) and runs while a barrier waits;
  // apply_faces adds the interface terms once the barrier has passed and the
  // neighbours' face data are published.
  double qloc[NV][DIM];
  auto apply_local = [&](double (&loc)[NV]) __attribute__((always_inline)) {
    for (int c = 0; c < NV; ++c) {
      const double* tile = &sx[(c * EPB + le) * NP];
      double xo = 0.0;
      if (act) {
        xo = tile[n];
        double gr[DIM];
        for (int d = 0; d < DIM; ++d) {
          const int st = L::stride(d);
          const double* row = &tile[n - ii[d] * st];
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < N1; ++k) s += sD[ii[d] * N1 + k] * row[k * st];
          gr[d] = g.rh2[d] * s;
        }
        double vg = 0.0;
        for (int j = 0; j < DIM; ++j) vg += cf.v[j] * gr[j];
        for (int d = 0; d < DIM; ++d) {
          qloc[c][d] = cw * cf.v[d] * vg + cf.nu * gr[d];
          sQ[(le * DIM + d) * NP + n] = jw * qloc[c][d];
        }
      }
      __syncthreads();
      double r = 0.0;
      if (act) {
        for (int d = 0; d < DIM; ++d) {
          const int st = L::stride(d);
          const double* row = &sQ[(le * DIM + d) * NP + n - ii[d] * st];
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < N1; ++k) s += sD[k * N1 + ii[d]] * row[k * st];
          r += g.rh2[d] * s;
        }
      }
      loc[c] = act ? jw * xo + a.dtm * r : 0.0;
      // sQ is rewritten next by apply_faces, after the barrier's own
      // __syncthreads; only a second component reuses it at once
      if (NV > 1) __syncthreads();
    }
  };
  auto apply_faces = [&](double (&out)[NV], const double (&loc)[NV]) __attribute__((always_inline)) {
    for (int c = 0; c < NV; ++c) {
      const double* tile = &sx[(c * EPB + le) * NP];
      double r = 0.0;
      if (act) {
        const double xo = tile[n];
        double Qd[DIM];
        for (int d = 0; d < DIM; ++d) Qd[d] = 0.0;
        for (int d = 0; d < DIM; ++d)
          for (int side = 0; side < 2; ++side) {
            if (ii[d] != (side ? P : 0)) continue;
            const double sgn = side ? 1.0 : -1.0;
            double xnb, qnb;
            face_vals(c, d, xnb, qnb);
            const double dow = cw * cf.v[d] * cf.v[d] + cf.nu;
            const double qn = 0.5 * sgn * (qloc[c][d] + qnb);
            const double tau = pen * fmax(dow, dnb[d][side]) * 0.5 * g.rh2[d];
            const double jump = xo - xnb;
            const double jfwf = g.J * g.rh2[d] * wn / sw[ii[d]];
            r += jfwf * (-qn + tau * jump);
            for (int d2 = 0; d2 < DIM; ++d2)
              Qd[d2] -= 0.5 * jfwf * jump * sgn * (cw * cf.v[d2] * cf.v[d] + (d2 == d ? cf.nu : 0.0));
          }
        for (int d = 0; d < DIM; ++d) sQ[(le * DIM + d) * NP + n] = Qd[d];
      }
      __syncthreads();
      if (act) {
        for (int d = 0; d < DIM; ++d) {
          const int st = L::stride(d);
          const double* row = &sQ[(le * DIM + d) * NP + n - ii[d] * st];
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < N1; ++k) s += sD[k * N1 + ii[d]] * row[k * st];
          r += g.rh2[d] * s;
        }
      }
      out[c] = act ? loc[c] + a.dtm * r : 0.0;
      // sQ is rewritten next by apply_local, after the __syncthreads of the
      // publish that precedes it (sx is read here at this thread's own node
      // only); only a second component reuses it at once
      if (NV > 1) __syncthreads();
    }
  };

  // vectors of the pipelined iteration (Ghysels-Vanroose, preconditioned)
  double x[NV], r[NV], u[NV], w[NV], m[NV], nn[NV], zv[NV], q[NV], s[NV], p[NV];
  for (int c = 0; c < NV; ++c) {
    x[c] = act ? a.x0[c * vs + own] : 0.0;
    zv[c] = q[c] = s[c] = p[c] = 0.0;
  }
  const double idg = act ? 1.0 / dg : 0.0;
  // the right-hand side, given or formed here from its terms (the same
  // arithmetic as k_lincomb, so both give the same bits)
  double bv[NV];
  double bb_l = 0.0;
  for (int c = 0; c < NV; ++c) {
    double bi = 0.0;
    if (act) {
      const long i = c * vs + own;
      if (a.b) {
        bi = a.b[i];
      } else {
        const double mwn = a.mw[n];
        for (int j = 0; j < a.bl.n; ++j) bi += a.bl.c[j] * (a.bl.m[j] ? mwn : 1.0) * a.bl.x[j][i];
      }
    }
    bv[c] = bi;
    bb_l += bi * bi;
  }
  // barrier records, double-buffered by barrier parity: a workgroup rewrites
  // its record of barrier k only at barrier k + 2, after every workgroup has
  // passed barrier k + 1 and so has finished reading the records of k
  auto rec = [&]() { return a.part + (long)(gen & 1u) * 16 * a.cap; };
  // barrier with one reduced value, the local part of the matvec of the
  // published vector into `loc` while it waits; advances the tag and the
  // face-buffer parity
  auto barrier1 = [&](const double (&v)[1], double (&tt)[1], double (&loc)[NV]) -> bool {
    const bool r = sync_reduce<1>(v, tt, rec(), a.cap, abort_w, a.tag0 + gen, a.spin_limit, &s_ok[(a.tag0 + gen) & 1u],
                                  [&]() __attribute__((always_inline)) {
                                    apply_local(loc);
                                    prefetch_faces();
                                  });
    gen += 1u;
    return r;
  };
  // r = b - A x and u = diag^-1 r (also used to replace the recurred
  // residual); the second barrier carries the face data of u together with
  // (r, r), so w = A u can follow (apply) without another barrier
  double wloc[NV];
  double bb = -1.0, thresh = 0.0;  // (b, b) and rtol^2 (b, b), from the first barrier
  auto true_residual = [&](double& rr_true) -> bool {
    const double z1[1] = {bb < 0.0 ? bb_l : 0.0};
    double t1[1];
    publish(x);
    if (!barrier1(z1, t1, wloc)) return false;
    if (bb < 0.0) {
      bb = t1[0];
      thresh = a.tol2 * bb;
    }
    apply_faces(w, wloc);
    double t_l = 0.0;
    for (int c = 0; c < NV; ++c) {
      r[c] = act ? bv[c] - w[c] : 0.0;
      u[c] = r[c] * idg;
      t_l += r[c] * r[c];
    }
    publish(u);
    const double v1[1] = {t_l};
    if (!barrier1(v1, t1, wloc)) return false;
    rr_true = t1[0];
    return true;
  };
  double rr0 = 0.0;
  bool ok = true_residual(rr0);
  if (ok) apply_faces(w, wloc);
  double gprev = 0.0, aprev = 0.0, rr = 0.0;
  int it = 0, replaced = 0;
  bool converged = false;
  while (ok) {
    // local (r,u), (w,u), (r,r); m = diag^-1 w; one barrier carries the face
    // data of m and the three sums
    double g_l = 0.0, d_l = 0.0, r_l = 0.0;
    for (int c = 0; c < NV; ++c) {
      g_l += r[c] * u[c];
      d_l += w[c] * u[c];
      r_l += r[c] * r[c];
      m[c] = w[c] * idg;
    }
    publish(m);
    const double v3[3] = {g_l, d_l, r_l};
    double tt[3];
    double nloc[NV];
    ok = sync_reduce<3>(v3, tt, rec(), a.cap, abort_w, a.tag0 + gen, a.spin_limit, &s_ok[(a.tag0 + gen) & 1u],
                        [&]() __attribute__((always_inline)) {
                          apply_local(nloc);
                          prefetch_faces();
                        });
    gen += 1u;
    if (!ok) break;
    const double gi = tt[0], di = tt[1];
    rr = tt[2];
    if (!(rr == rr)) break;
    if (rr <= thresh) {
      // confirm with the true residual; replace the recurred one if it misses
      ok = true_residual(rr);
      if (!ok) break;
      if (rr <= thresh) { converged = true; break; }
      // restart the recurrences from the true residual (at most 3 times)
      if (++replaced > 3 || it >= a.maxit) break;
      apply_faces(w, wloc);
      for (int c = 0; c < NV; ++c) zv[c] = q[c] = s[c] = p[c] = 0.0;
      gprev = 0.0;
      aprev = 0.0;
      continue;
    }
    if (it >= a.maxit) break;
    apply_faces(nn, nloc);  // n = A m: the face terms (neighbour data published before the barrier)
    double beta = 0.0, alpha;
    if (gprev == 0.0) {
      alpha = gi / di;
    } else {
      beta = gi / gprev;
      alpha = gi / (di - beta * gi / aprev);
    }
    gprev = gi;
    aprev = alpha;
    for (int c = 0; c < NV; ++c) {
      zv[c] = nn[c] + beta * zv[c];
      q[c] = m[c] + beta * q[c];
      s[c] = w[c] + beta * s[c];
      p[c] = u[c] + beta * p[c];
      x[c] += alpha * p[c];
      r[c] -= alpha * s[c];
      u[c] -= alpha * q[c];
      w[c] -= alpha * zv[c];
    }
    ++it;
  }
  if (act)
    for (int c = 0; c < NV; ++c) a.x[c * vs + own] = x[c];
  if (blockIdx.x == 0 && t == 0) {
    a.res->rr = rr;
    a.res->bb = bb;
    a.res->thresh = thresh;
    a.res->it = it;
    a.res->it_last = ok ? (converged ? 2 : 0) : -1;  // 2: converged, 0: not converged, -1: aborted
  }
}

template <int DIM, int P, int NV>
static hipError_t pcg_dim_p_nv(const PCGArgs& a, const CoefP& cf, const Geo& g, const double* tab, int max_blocks,
                               bool cooperative, hipStream_t s) {
  using L = PT<DIM, P>;
  const int nb = (g.E + L::EPB - 1) / L::EPB;
  if (nb > max_blocks || nb > a.cap) return hipErrorCooperativeLaunchTooLarge;
  PCGArgs aa = a;
  CoefP cc = cf;
  Geo gg = g;
  const double* tt = tab;
  if (!cooperative) {  // ordinary launch: the grid fits the device at once (nb <= max_blocks)
    hipLaunchKernelGGL((k_pcg_persistent<DIM, P, NV>), dim3(nb), dim3(L::NT), 0, s, aa, cc, gg, tt);
    return hipGetLastError();
  }
  void* args[] = {&aa, &cc, &gg, &tt};
  return hipLaunchCooperativeKernel((const void*)k_pcg_persistent<DIM, P, NV>, dim3(nb), dim3(L::NT), args, 0, s);
}

template <int DIM, int P>
static hipError_t pcg_dim_p(const PCGArgs& a, int nv, const CoefP& cf, const Geo& g, const double* tab,
                            int max_blocks, bool cooperative, hipStream_t s) {
  if (nv == 1) return pcg_dim_p_nv<DIM, P, 1>(a, cf, g, tab, max_blocks, cooperative, s);
  return hipErrorInvalidValue;  // systems use the multi-kernel PCG (faster there)
}

template <int DIM, int P, int NV>
static int occ_dim_p_nv() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_pcg_persistent<DIM, P, NV>,
                                                   PT<DIM, P>::NT, 0) != hipSuccess)
    return 0;
  return per_cu;
}

template <int DIM, int P>
static int occ_dim_p(int nv) {
  if (nv == 1) return occ_dim_p_nv<DIM, P, 1>();
  return 0;
}

#define SISDC_PDISPATCH(P_, BODY)                    \
  switch (P_) {                                      \
    case 1: { constexpr int PP = 1; BODY; } break;  \
    case 2: { constexpr int PP = 2; BODY; } break;  \
    case 3: { constexpr int PP = 3; BODY; } break;  \
    case 4: { constexpr int PP = 4; BODY; } break;  \
    case 5: { constexpr int PP = 5; BODY; } break;  \
    case 6: { constexpr int PP = 6; BODY; } break;  \
    case 7: { constexpr int PP = 7; BODY; } break;  \
    case 8: { constexpr int PP = 8; BODY; } break;  \
    default: break;                                  \
  }

hipError_t launch_pcg_persistent(const PCGArgs& a, int nv, const CoefP& cf, const Geo& g, const double* tab,
                                 int max_blocks, bool cooperative, hipStream_t s) {
  if (g.dim == 2) { SISDC_PDISPATCH(g.P, return (pcg_dim_p<2, PP>(a, nv, cf, g, tab, max_blocks, cooperative, s))); }
  if (g.dim == 3) { SISDC_PDISPATCH(g.P, return (pcg_dim_p<3, PP>(a, nv, cf, g, tab, max_blocks, cooperative, s))); }
  return hipErrorInvalidValue;
}

// Workgroups of one persistent launch on this geometry (one per tile).
int pcg_persistent_grid(const Geo& g) {
  if (g.dim == 2) { SISDC_PDISPATCH(g.P, return ((g.E + PT<2, PP>::EPB - 1) / PT<2, PP>::EPB)); }
  if (g.dim == 3) { SISDC_PDISPATCH(g.P, return ((g.E + PT<3, PP>::EPB - 1) / PT<3, PP>::EPB)); }
  return 0;
}

int pcg_persistent_blocks_per_cu(const Geo& g, int nv) {
  if (g.dim == 2) { SISDC_PDISPATCH(g.P, return (occ_dim_p<2, PP>(nv))); }
  if (g.dim == 3) { SISDC_PDISPATCH(g.P, return (occ_dim_p<3, PP>(nv))); }
  return 0;
}

}  // namespace sisdc
