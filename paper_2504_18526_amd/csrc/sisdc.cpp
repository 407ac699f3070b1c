// libsisdc host side: level storage, the SI-SDC sweep, the FAS V-cycle and the
// start strategies, the Jacobi-PCG driver, and the C ABI of include/sisdc.h.
//
// Method (arXiv 2504.18526): incremental SI(1)/SI(2) predictor and corrector
// (Sec. 3), FAS multilevel SDC with transfers I, P, R = I^T, V-cycle and the
// cascade / FMG starts (Sec. 4, Alg. 1-4), DG-SEM in space (Sec. 6).  Every
// vector lives in device memory; the host only sequences kernel launches and
// reads back the CG convergence flag once per batch of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/sisdc.h"
#include "common.hpp"
#include "launch.hpp"
#include "mlp.hpp"
#include "scratch.hpp"
#include "tables.hpp"

using namespace sisdc;

namespace {

// Thrown where a step under capture would need the host (a wait for the GPU);
// the capture is dropped and the step runs without a graph.
struct CaptureNeedsHost {};

thread_local std::string g_last_error;

struct Err {
  int code;
  std::string msg;
};

#define HIPCHECK(x)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) throw Err{SISDC_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

void fail(int code, const std::string& m) { throw Err{code, m}; }

float* falloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(&p, n * sizeof(float)) != hipSuccess) fail(SISDC_ENOMEM, "hipMalloc failed");
  return (float*)p;
}

double* dalloc(size_t n) {
  void* p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) fail(SISDC_ENOMEM, "hipMalloc failed");
  return (double*)p;
}

struct Level {
  int P = 0, M = 0, n1 = 0, np = 0, E = 0, nv = 0;
  long vs = 0, vlen = 0;
  Geo g{};
  std::vector<double> xg, wg, D, tau, dtau, wnn;
  double* tab = nullptr;  // D (n1*n1) then w (n1)
  double* mw = nullptr;   // J w per node (np)
  double* u = nullptr;    // (M+1) x vlen
  double* unew = nullptr; // (M+1) x vlen
  double* f = nullptr;    // M x vlen, f(u_m), m = 1..M
  double* C = nullptr;    // (M+1) x vlen, C(u_m), m = 0..M
  double* Cnew = nullptr; // (M+1) x vlen
  double* X = nullptr;    // M x vlen, K_{D(u_{m-1})} u_m
  double* gf = nullptr;   // M x vlen, FAS right-hand side
  double* v = nullptr;    // (M+1) x vlen, projected fine iterate
  double* r = nullptr;    // M x vlen, residual
  double* q = nullptr;    // M x vlen, quadrature
  double *b = nullptr, *y = nullptr, *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
  double* idg = nullptr;        // NP-periodic inverse Jacobi diagonal (isotropic path)
  double *diag = nullptr, *cr = nullptr, *cz = nullptr, *cp = nullptr, *cs = nullptr, *cw = nullptr;
  double* trace = nullptr;
  unsigned long long* fz = nullptr;  // tagged face values of the persistent PCG (2 buffers, 2 words each)
  unsigned long long* ft = nullptr;  // tagged face traces of the persistent PCG (2 buffers, 2 words each)
  size_t fwords = 0;                 // words of fz and of ft
  bool persistent = false;     // solves run as one persistent launch
  // FP32 copies and work vectors of the mixed-precision inner solves
  float* tab32 = nullptr;
  float *ub32 = nullptr, *r32 = nullptr, *e32 = nullptr, *cr32 = nullptr, *cz32 = nullptr, *cp32 = nullptr,
        *cs32 = nullptr, *cw32 = nullptr, *diag32 = nullptr, *trace32 = nullptr;
  float* idg32 = nullptr;
  // Inverse Jacobi diagonals of the isotropic solves, by (dt_m, nu, C_tau):
  // the same few recur within a time step (both stages of a node, every
  // sweep), and each is formed once.
  struct IdgCache {
    static constexpr int kSlots = 8;
    void* tab = nullptr;  // kSlots tables of NP values
    double key[kSlots][3] = {};
    int n = 0, next = 0;
  } idgc64, idgc32;
  // learned initial guess (element-local MLP), see sisdc_net_*
  struct Net {
    bool on = false;          // initialised
    bool use = false;         // apply before every solve of this level
    bool harvest = false;     // record (r0, x* - x0) rows of every solve
    MlpShape sh{};
    float *theta = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    int max_batch = 0, max_rows = 0, rows = 0, step = 0;
    float *Xd = nullptr, *Td = nullptr;                          // harvested rows
    float *Z1 = nullptr, *A1 = nullptr, *Z2 = nullptr, *A2 = nullptr, *Y = nullptr, *dY = nullptr,
          *dA = nullptr, *dZ = nullptr;                          // training work (max_batch rows)
    float *Xi = nullptr, *A1i = nullptr, *A2i = nullptr, *Yi = nullptr;  // inference work (E * nv rows)
    double *nrm = nullptr, *xnew = nullptr, *x0h = nullptr, *r0h = nullptr;
    float *Xs = nullptr, *Ts = nullptr;                          // staging of caller rows
    double* lossp = nullptr;                                     // loss partials, 64 per batch
    int loss_cap = 0;                                            // batches the loss buffer holds
  } net;
  double mass_total = 0.0;  // 1^T M 1 of one component: E times the sum of the element's mass weights
  double* fds = nullptr;    // fast-diagonalisation tables of the element block (S_d, lam_d per axis)
  bool stale = true;
  double stored_dt = -1.0;
  bool has_g = false;
  int last_iters = 8;
  double* um(int m) const { return u + (long)m * vlen; }
  double* unm(int m) const { return unew + (long)m * vlen; }
};

struct Transfer {  // between level i (fine) and i+1 (coarse)
  bool h = false;        // 2:1 h-coarsened: Ix is (2 n1f x n1c), Px and Rx (n1c x 2 n1f) on a pair of
                         // fine elements per axis (left child first)
  double* Ix = nullptr;  // (n1f x n1c) coarse -> fine
  double* Px = nullptr;  // (n1c x n1f) fine -> coarse
  double* Rx = nullptr;  // (n1c x n1f) = Ix^T
  std::vector<double> It, Pt;  // It: (Mf x Mc), Pt: (Mc x Mf)
  std::vector<double> Rt;      // (Mc x Mf) time restriction of residuals: I_t^T, or
                               // C_c^-1 I_t^T C_f for the non-incremental form
};

}  // namespace

// Offset of the convergence word behind the result record, in the device
// block that holds both and in their pinned host mirror.
constexpr size_t kDoneOffset = 128;
static_assert(sizeof(CGRes) <= kDoneOffset, "the result record fits before the convergence word");

struct sisdc_handle {
  sisdc_problem prob{};
  sisdc_method meth{};
  hipStream_t stream = nullptr;
  int dev = 0;              // device current at creation
  bool registered = false;  // stream entered in the persistent-solve order
  int lane = -1;            // host thread of the batch step running this handle (-1: none)
  int lanes = 0;            // host threads of that batch step
  // step graph (sisdc_set_graph): the whole step captured once and replayed
  bool graph_on = false;
  bool capturing = false;           // a step is being captured on `stream`
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr; // stream the step is captured on (the handle's own may be the null stream)
  double g_dt = 0.0;                // step size and solver form the graph was captured with
  int g_form = -1;
  int g_refused_form = -1;          // form whose capture needed the host (not tried again)
  double g_refused_dt = 0.0;
  std::vector<std::pair<int, int>> g_ring_meta;  // result records the graph writes
  sisdc_stats g_st{};               // host-side counts of one captured step
  long long g_captures = 0, g_replays = 0;
  bool g_last = false;              // the last step ran through the graph
  EqP eq{};
  std::vector<Level> lv;
  std::vector<Transfer> tr;
  double* partials = nullptr;  // CG partial sums: gam (3 cap), rr (2 cap), del, bbp (cap each)
  double* cons = nullptr;      // partial sums of the conservation correction fused into the isotropic PCG
  double* alpha = nullptr;     // 2 CG step lengths
  float* partials32 = nullptr; // FP32 CG partial sums (7 cap)
  float* alpha32 = nullptr;
  double* ir_tot = nullptr;    // (r,r), (b,b) of the FP64 residual of iterative refinement
  double* gtot = nullptr;      // (delta, r0), (delta, A delta) of a learned guess
  int* nrej = nullptr;         // learned guesses rejected (device counter)
  int* hnrej = nullptr;        // pinned mirror
  int nrej_seen = 0;
  double* hir_tot = nullptr;   // pinned mirror
  int* done_gen = nullptr;     // id of the last converged solve
  CGRes* res = nullptr;        // device result record
  CGRes* hres = nullptr;       // pinned host mirror of res ...
  int* hdone = nullptr;        // ... and of done_gen
  int solve_id = 0;
  // persistent PCG
  unsigned long long* ppart = nullptr;  // barrier records of the persistent PCG (2 x 16 x pcap words)
  unsigned tag = 0;                     // last barrier tag handed out
  int pcap = 0;
  unsigned* bar = nullptr;     // grid barrier words
  CGRes* ring = nullptr;       // result records of solves not yet collected
  CGRes* hring = nullptr;      // pinned host mirror
  int ring_n = 0;              // records in flight
  std::vector<std::pair<int, int>> ring_meta;  // (level, maxit) per record
  // event timing of the persistent PCG launches (sisdc_pcg_timing)
  bool ptime = false;
  std::vector<hipEvent_t> pev;   // 2 per ring record: before / after the launch
  std::vector<char> ring_timed;  // per record: events recorded
  std::vector<double> pt_us;     // per level: summed event time (us) ...
  std::vector<long long> pt_n, pt_it;  // ... launches and iterations
  // event timing of the multi-kernel PCG's launches (sisdc_cg_kernel_timing_get):
  // per level and kernel (2 level + 0: vector update, 2 level + 1: matvec),
  // the launches that did a full iteration's work and their summed event time
  std::vector<hipEvent_t> mev;   // pool: 3 events per iteration of a chunk
  std::vector<double> kt_us;
  std::vector<long long> kt_n;
  int kt_stride = 1;             // time every kt_stride-th multi-kernel solve
  long long kt_solves = 0;       // multi-kernel solves since timing was switched on
  double* lam_dev = nullptr;
  double* hlam = nullptr;      // pinned
  double* state = nullptr;
  double* io = nullptr;      // staging for host pointers, (Mmax+1) x vlen_max
  // artificial viscosity (method av_c > 0): eps per element, the same on
  // every level; the fine level's discrete Legendre transform
  bool av = false;
  double* eps = nullptr;
  double* av_tab = nullptr;
  size_t io_len = 0;
  double lam = 0.0;
  double visc = 0.0;           // viscous bound added to kappa_m (NS)
  bool have_state = false;
  double ctau = 2.0;
  sisdc_stats st{};
};

namespace {

// ------------------------------------------------------------------ helpers
void lincomb(sisdc_handle* h, const Level& L, double* out, std::initializer_list<std::pair<double, const double*>> terms,
             std::initializer_list<int> mflags = {}) {
  LinComb lc{};
  int k = 0;
  auto mit = mflags.begin();
  for (auto& t : terms) {
    if (k >= 8) fail(SISDC_EINVAL, "lincomb: too many terms");
    lc.x[k] = t.second;
    lc.c[k] = t.first;
    lc.m[k] = (mit != mflags.end()) ? *mit++ : 0;
    ++k;
  }
  lc.n = k;
  HIPCHECK(launch_lincomb(out, lc, L.vlen, L.mw, L.np, h->stream));
}

LinComb make_lc(std::initializer_list<std::pair<double, const double*>> terms, std::initializer_list<int> mflags) {
  LinComb lc{};
  int k = 0;
  auto mit = mflags.begin();
  for (auto& t : terms) {
    if (k >= 8) fail(SISDC_EINVAL, "lincomb: too many terms");
    lc.x[k] = t.second;
    lc.c[k] = t.first;
    lc.m[k] = (mit != mflags.end()) ? *mit++ : 0;
    ++k;
  }
  lc.n = k;
  return lc;
}

void lincomb_v(sisdc_handle* h, const Level& L, double* out, const std::vector<double>& c,
               const std::vector<const double*>& x, const std::vector<int>& m) {
  // chunks of 8 terms: out = sum; later chunks accumulate onto out
  size_t i = 0;
  bool first = true;
  while (i < c.size() || first) {
    LinComb lc{};
    int k = 0;
    if (!first) {
      lc.x[0] = out;
      lc.c[0] = 1.0;
      lc.m[0] = 0;
      k = 1;
    }
    while (k < 8 && i < c.size()) {
      lc.x[k] = x[i];
      lc.c[k] = c[i];
      lc.m[k] = m.empty() ? 0 : m[i];
      ++k;
      ++i;
    }
    lc.n = k;
    HIPCHECK(launch_lincomb(out, lc, L.vlen, L.mw, L.np, h->stream));
    first = false;
  }
}

void copy_d2d(sisdc_handle* h, double* dst, const double* src, long n) {
  if (h->capturing) {
    HIPCHECK(launch_copy(src, dst, n, h->stream));
    return;
  }
  HIPCHECK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
}

template <typename T>
void copy_any(sisdc_handle* h, T* dst, const T* src, long n) {
  if (h->capturing) throw CaptureNeedsHost{};
  HIPCHECK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, h->stream));
}

CoefP coef_for(sisdc_handle* h, const Level& L, double dtm, const double* ub) {
  CoefP c{};
  c.eps = h->av ? h->eps : nullptr;  // the artificial viscosity joins the diffusion
  if (h->meth.integrator == SISDC_IMEX_EULER) {  // eq. H_IMEX: A_d alone
    c.nu = (h->eq.eq == EQ_EULER || h->eq.eq == EQ_NS) ? 0.0 : h->eq.nu;
    (void)L;
    (void)ub;
    return c;
  }
  switch (h->eq.eq) {
    case EQ_CONVDIFF:
      c.c = 0.5 * dtm;
      for (int d = 0; d < 3; ++d) c.v[d] = h->eq.a[d];
      c.nu = h->eq.nu;
      c.ub = nullptr;
      break;
    case EQ_BURGERS:
      c.c = 0.5 * dtm;
      for (int d = 0; d < 3; ++d) c.v[d] = 1.0;
      c.nu = h->eq.nu;
      c.ub = ub;
      break;
    default:  // systems: kappa_m I, kappa_m = (dt_m / 2) lam*^2 (+ viscous bound, NS)
      c.c = 0.0;
      c.nu = 0.5 * dtm * h->lam * h->lam + h->visc;
      c.ub = nullptr;
  }
  (void)L;
  return c;
}

// The physical diffusion nu I (+ eps_e I) of F's diffusive term.
CoefP coef_nu(sisdc_handle* h) {
  CoefP c{};
  c.nu = h->eq.nu;
  c.eps = h->av ? h->eps : nullptr;
  return c;
}

void conv(sisdc_handle* h, const Level& L, const double* in, double* out, int nodes = 1) {
  HIPCHECK(launch_conv(in, out, L.g, h->eq, L.tab, h->stream, nodes));
}

void sipg(sisdc_handle* h, const Level& L, const CoefP& cf, const double* x, double* out, double alpha,
          double beta) {
  HIPCHECK(launch_sipg(x, out, L.nv, cf, L.trace, alpha, beta, h->ctau, L.g, L.tab, h->stream));
}

bool is_system(const sisdc_handle* h) { return h->eq.eq == EQ_EULER || h->eq.eq == EQ_NS; }
bool has_physical_diffusion(sisdc_handle* h) { return !is_system(h) && (h->eq.nu != 0.0 || h->av); }

// f = F(u) = C(u) - K_nu u (scalars), C(u) (Euler), C(u) + V(u) (NS); with
// artificial viscosity nu + eps_e in the scalars' term and - K_eps u added
// for systems; Cu = C(u) precomputed
void frhs_from_c(sisdc_handle* h, const Level& L, const double* u, const double* Cu, double* f) {
  if (h->av && is_system(h)) {
    if (h->eq.eq == EQ_NS && h->eq.mu != 0.0)
      HIPCHECK(launch_visc(u, Cu, f, L.trace, L.g, h->eq, L.tab, h->stream));
    else if (f != Cu)
      copy_d2d(h, f, Cu, L.vlen);
    CoefP ce{};
    ce.eps = h->eps;
    sipg(h, L, ce, u, L.t3, 0.0, 1.0);
    lincomb(h, L, f, {{1.0, f}, {-1.0, L.t3}});
    return;
  }
  if (has_physical_diffusion(h)) {
    // quadrilaterals: f = C - K_nu u in one pass of the isotropic kernel
    if (L.g.dim == 2 && f != Cu && launch_sipg_iso2_add(u, Cu, f, L.nv, coef_nu(h), 0.0, -1.0, h->ctau, L.g, L.tab, h->stream) ==
                            hipSuccess)
      return;
    (void)hipGetLastError();
    sipg(h, L, coef_nu(h), u, L.t3, 0.0, 1.0);
    lincomb(h, L, f, {{1.0, Cu}, {-1.0, L.t3}});
    return;
  }
  if (h->eq.eq == EQ_NS && h->eq.mu != 0.0) {
    HIPCHECK(launch_visc(u, Cu, f, L.trace, L.g, h->eq, L.tab, h->stream));  // f = C(u) + V(u), no copy
    return;
  }
  if (f != Cu) copy_d2d(h, f, Cu, L.vlen);
}

// ------------------------------------------------------------------ PCG
// Work buffers of one precision for the multi-kernel PCG.
template <typename T>
struct CGBufs {
  T *r, *z, *p, *s, *w, *diag, *trace;
  const T* tab;
  T* partials;
  T* alpha;
  T* idg;
  int* done_gen;  // id of the last converged solve
  CGRes* res;     // result record
  T* cons;        // partial sums of the fused conservation correction (NULL: none)
};

CGBufs<double> bufs64(sisdc_handle* h, Level& L) {
  return CGBufs<double>{L.cr,       L.cz,     L.cp,  L.cs,        L.cw,  L.diag, L.trace,
                        L.tab,      h->partials, h->alpha, L.idg, h->done_gen, h->res, h->cons};
}

CGBufs<float> bufs32(sisdc_handle* h, Level& L) {
  return CGBufs<float>{L.cr32, L.cz32,        L.cp32,      L.cs32, L.cw32,      L.diag32, L.trace32,
                       L.tab32, h->partials32, h->alpha32, L.idg32, h->done_gen, h->res, nullptr};
}

template <typename T>
CGStateT<T> cg_state(sisdc_handle* h, const CGBufs<T>& B, const T* b, T* x, double rtol) {
  CGStateT<T> cg{};
  cg.x = x;
  cg.r = B.r;
  cg.z = B.z;
  cg.p = B.p;
  cg.s = B.s;
  cg.w = B.w;
  cg.trace = B.trace;
  cg.b = b;
  cg.x0 = nullptr;
  cg.zs = nullptr;
  cg.cons = nullptr;
  cg.diag = B.diag;
  cg.cap = kElemCap;
  cg.gam = B.partials;
  cg.rr = B.partials + 3 * kElemCap;
  cg.del = B.partials + 5 * kElemCap;
  cg.bbp = B.partials + 6 * kElemCap;
  cg.alpha = B.alpha;
  cg.done_gen = B.done_gen;
  cg.res = B.res;
  cg.tol2 = (T)(rtol * rtol);
  return cg;
}

// Jacobi-PCG (Chronopoulos-Gear form) on M + dt_m K_D; x holds the initial
// guess on entry.  Iterations are enqueued in batches; the host reads the
// convergence record once per batch.
constexpr int kRing = 2048;
constexpr double kPersistentMinRtol = 1e-11;
constexpr long kSpinLimit = 1L << 21;

void account(sisdc_handle* h, int iters, bool converged, double rel) {
  h->st.solves += 1;
  h->st.cg_iters += iters;
  h->st.cg_iters_max = std::max(h->st.cg_iters_max, iters);
  h->st.max_rel_residual = std::max(h->st.max_rel_residual, rel);
  if (!converged) h->st.not_converged += 1;
}

// Conservation correction after a solve (method option `conserve`): shift
// every component of x by a constant so that 1^T M x = 1^T b, which the
// exact solution satisfies (the SIPG operator annihilates constants and is
// symmetric); an iterative solve leaves 1^T (b - A x) of the order of its
// tolerance, and the shift removes it, so the totals the method conserves
// hold to round-off whatever the tolerance.
// On the streaming isotropic PCG the shift can instead be fused into the
// solve (running sums in every update kernel): that pays on large levels,
// where the update is bandwidth-bound and the sums ride along, but on small
// ones the sums' block reductions cost more per iteration than the two
// passes after the solve (three-level Euler workload: 39.2 against 33.4 ms
// per step with every level fused).
constexpr long kFusedConserveMin = 1L << 21;  // values per vector
bool fused_conserve(const sisdc_handle* h, const Level& L) {
  return h->meth.conserve && L.vlen >= kFusedConserveMin;
}

void conserve_fix(sisdc_handle* h, Level& L, const double* b, const LinComb* bl, double* x) {
  if (!h->meth.conserve) return;
  HIPCHECK(launch_conserve(b, bl, x, L.nv, L.vs, L.mw, L.np, L.mass_total, h->partials, 7 * kElemCap, h->stream));
}

// Collect the result records of persistent solves enqueued since the last
// collection (one stream synchronisation).
void drain_rejections(sisdc_handle* h) {
  if (h->capturing) throw CaptureNeedsHost{};
  HIPCHECK(hipMemcpyAsync(h->hnrej, h->nrej, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  h->st.net_rejected += *h->hnrej - h->nrej_seen;
  h->nrej_seen = *h->hnrej;
}

void drain(sisdc_handle* h) {
  if (h->capturing) throw CaptureNeedsHost{};
  if (h->st.net_guesses > 0) drain_rejections(h);
  if (h->ring_n == 0) return;
  HIPCHECK(hipMemcpyAsync(h->hring, h->ring, h->ring_n * sizeof(CGRes), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  bool aborted = false, nonfinite = false;
  for (int i = 0; i < h->ring_n; ++i) {
    const CGRes& r = h->hring[i];
    if (r.it_last < 0) aborted = true;
    const bool conv = (r.it_last & 2) != 0;
    const double rel = r.bb > 0.0 ? std::sqrt(r.rr / r.bb) : 0.0;
    if (!std::isfinite(rel) || !std::isfinite(r.rr) || !std::isfinite(r.bb)) nonfinite = true;
    account(h, r.it, conv, rel);
    const int li = h->ring_meta[i].first;
    Level& L = h->lv[li];
    L.last_iters = std::max(1, r.it);
    if (h->ring_timed[i]) {
      float ms = 0.0f;
      HIPCHECK(hipEventElapsedTime(&ms, h->pev[2 * i], h->pev[2 * i + 1]));
      h->pt_us[li] += 1000.0 * ms;
      h->pt_n[li] += 1;
      h->pt_it[li] += r.it;
    }
  }
  h->ring_n = 0;
  h->ring_meta.clear();
  h->ring_timed.clear();
  if (aborted) {
    HIPCHECK(hipMemsetAsync(h->bar, 0, 512, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    for (auto& L : h->lv) L.persistent = false;
    fail(SISDC_EDEVICE, "persistent PCG barrier timed out; persistent solves disabled for this handle");
  }
  if (nonfinite) fail(SISDC_ENONFINITE, "non-finite residual in the Helmholtz solve");
}

// Levels that use the persistent PCG under SISDC_CG_AUTO: scalar equations
// whose tiles fit the partial-sum records.  For systems the per-workgroup
// work of an iteration grows with the number of components and the
// multi-kernel form is faster (three-level Euler workload: 54 against 84 ms
// per step).
bool persistent_fits(const sisdc_handle* h, const Level& L, int variant) {
  return (variant == SISDC_CG_AUTO || variant == SISDC_CG_PERSISTENT_COOPERATIVE) && L.nv == 1 && !h->av &&
         elem_tile_count(L.g) <= h->pcap;
}

// Order of the persistent solves on one device.  A persistent grid relies on
// all its workgroups being resident together, so two must never compete for
// the device: a solve launched on one stream waits (on the GPU) for the
// latest persistent solve launched on another.  Every handle registers its
// stream here.  While one stream is registered, stream order alone does
// this and no event is recorded; with several, an event recorded after
// each launch marks it (a launch made before the second stream appeared is
// marked when first needed, by an event recorded on its stream then).
//
// Lanes: the host threads of a batch step (lane = thread).  A lane's solve
// whose grid is at most 1/(lanes + 1) of the workgroups the device holds at
// once may overlap the solves of the other lanes (at most `lanes` of them
// run at a time, each thread stepping one instance at a time, and together
// they fit on the device); it still waits for the latest ordinary launch,
// and an ordinary launch waits for the latest solve of every lane.
struct PersistentOrder {
  std::mutex m;
  std::vector<std::pair<hipStream_t, int>> streams;  // streams of live handles, with handle counts
  hipEvent_t done = nullptr;
  hipStream_t last = nullptr;  // stream of the latest persistent launch
  bool pending = false;        // that launch may still be running
  bool marked = false;         // `done` was recorded after it
  std::vector<hipEvent_t> lane_ev;      // recorded after the latest overlapping solve of each lane
  std::vector<hipStream_t> lane_last;   // its stream; null once an ordinary launch has waited for it
};
constexpr int kMaxDevices = 64;
PersistentOrder g_porder[kMaxDevices];

PersistentOrder& porder(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(SISDC_EDEVICE, "device ordinal out of range");
  return g_porder[dev];
}

void porder_register(int dev, hipStream_t s) {
  PersistentOrder& po = porder(dev);
  std::lock_guard<std::mutex> lock(po.m);
  for (auto& e : po.streams)
    if (e.first == s) {
      e.second += 1;
      return;
    }
  po.streams.emplace_back(s, 1);
}

// The caller has synchronised the device: nothing of `s` is still running.
void porder_unregister(int dev, hipStream_t s) {
  if (dev < 0 || dev >= kMaxDevices) return;
  PersistentOrder& po = g_porder[dev];
  std::lock_guard<std::mutex> lock(po.m);
  for (size_t i = 0; i < po.streams.size(); ++i)
    if (po.streams[i].first == s) {
      if (--po.streams[i].second == 0) po.streams.erase(po.streams.begin() + (long)i);
      break;
    }
  if (po.pending && po.last == s) po.pending = false;
  for (auto& ls : po.lane_last)
    if (ls == s) ls = nullptr;
  // the last handle of the device is gone: release the ordering events, so no
  // HIP object of the library outlives its handles
  if (po.streams.empty()) {
    if (po.done) (void)hipEventDestroy(po.done);
    for (hipEvent_t e : po.lane_ev)
      if (e) (void)hipEventDestroy(e);
    po.lane_ev.clear();
    po.lane_last.clear();
    po.done = nullptr;
    po.pending = false;
    po.marked = false;
    po.last = nullptr;
  }
}

// Whether a lane's persistent launch on level L may overlap those of the
// other lanes: its grid is at most 1/(lanes + 1) of the workgroups the
// device holds at once.
bool lane_may_overlap(const sisdc_handle* h, const Level& L) {
  if (h->lane < 0) return false;
  int ncu = 0;
  HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->dev));
  const long max_blocks = (long)pcg_persistent_blocks_per_cu(L.g, L.nv) * ncu;
  return (long)pcg_persistent_grid(L.g) * (h->lanes + 1) <= max_blocks;
}

// Ordering of one persistent launch (or of a captured step holding them) on
// h's stream against the persistent launches of other streams; po.m held.
void porder_before(PersistentOrder& po, sisdc_handle* h, bool overlap) {
  if (po.streams.size() <= 1) return;
  if (!po.done) HIPCHECK(hipEventCreateWithFlags(&po.done, hipEventDisableTiming));
  if (po.pending && po.last != h->stream) {
    if (!po.marked) HIPCHECK(hipEventRecord(po.done, po.last));
    po.marked = true;
    HIPCHECK(hipStreamWaitEvent(h->stream, po.done, 0));
  }
  if (!overlap)
    for (size_t l = 0; l < po.lane_last.size(); ++l)
      if (po.lane_last[l] && po.lane_last[l] != h->stream) {
        HIPCHECK(hipStreamWaitEvent(h->stream, po.lane_ev[l], 0));
        po.lane_last[l] = nullptr;
      }
}

void porder_after(PersistentOrder& po, sisdc_handle* h, bool overlap) {
  const bool several = po.streams.size() > 1;
  if (overlap && several) {
    if (po.lane_ev.size() <= (size_t)h->lane) {
      po.lane_ev.resize(h->lane + 1, nullptr);
      po.lane_last.resize(h->lane + 1, nullptr);
    }
    if (!po.lane_ev[h->lane]) HIPCHECK(hipEventCreateWithFlags(&po.lane_ev[h->lane], hipEventDisableTiming));
    HIPCHECK(hipEventRecord(po.lane_ev[h->lane], h->stream));
    po.lane_last[h->lane] = h->stream;
    return;
  }
  po.last = h->stream;
  po.pending = true;
  po.marked = false;
  if (several) {
    HIPCHECK(hipEventRecord(po.done, h->stream));
    po.marked = true;
  }
}

// Zero every tagged word of the persistent PCG (barrier records, and the face
// records of every level), so that no tag handed out afterwards from 1 on
// can match a word written before.
void clear_tagged_records(sisdc_handle* h) {
  HIPCHECK(launch_zero_scratch(h->ppart, (size_t)2 * 16 * h->pcap * sizeof(unsigned long long), h->stream));
  for (auto& L : h->lv)
    if (L.fz) {
      HIPCHECK(launch_zero_scratch(L.fz, L.fwords * sizeof(unsigned long long), h->stream));
      HIPCHECK(launch_zero_scratch(L.ft, L.fwords * sizeof(unsigned long long), h->stream));
    }
}

// b null: the kernel forms the right-hand side from `bl`.
bool persistent_solve(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, double* x,
                      double rtol, int maxit, const double* x0 = nullptr, const LinComb* bl = nullptr) {
  if (!b && !bl) fail(SISDC_EINVAL, "internal: no right-hand side");
  if (h->ring_n >= kRing) drain(h);
  PCGArgs a{};
  a.b = b;
  if (!b) {
    a.bl = *bl;
    a.mw = L.mw;
  }
  a.x = x;
  a.x0 = x0 ? x0 : x;
  a.fz = L.fz;
  a.ft = L.ft;
  a.part = h->ppart;
  a.bar = h->bar;
  a.res = h->ring + h->ring_n;
  a.tol2 = rtol * rtol;
  a.dtm = dtm;
  a.ctau = h->ctau;
  a.maxit = maxit;
  a.cap = h->pcap;
  a.spin_limit = kSpinLimit;
  // more tags than a launch can use (2 + maxit + 2 per residual check, at most 4 checks); when the
  // 32-bit tags run out the records are cleared (tag 0) and the count starts again
  const unsigned long long need = 2ull * (unsigned long long)maxit + 64ull;
  if (need > 0x40000000ull) return false;  // such an iteration cap takes the multi-kernel form
  if ((unsigned long long)h->tag + need >= 0xffffffffull) {
    if (h->capturing) throw CaptureNeedsHost{};
    clear_tagged_records(h);
    h->tag = 0;
  }
  a.tag0 = h->tag + 1u;
  h->tag += (unsigned)need;
  int dev = 0, ncu = 0;
  HIPCHECK(hipGetDevice(&dev));
  HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int max_blocks = pcg_persistent_blocks_per_cu(L.g, L.nv) * ncu;
  const int slot = h->ring_n;
  const bool cooperative = h->meth.cg_variant == SISDC_CG_PERSISTENT_COOPERATIVE;
  // a lane's solve small enough to share the device with the other lanes
  const bool overlap = !cooperative && lane_may_overlap(h, L);
  PersistentOrder& po = porder(h->dev);
  std::unique_lock<std::mutex> lock(po.m, std::defer_lock);
  if (!h->capturing) {  // a captured step is ordered as a whole when it is launched
    lock.lock();
    porder_before(po, h, overlap);
  }
  if (h->ptime) HIPCHECK(hipEventRecord(h->pev[2 * slot], h->stream));
  hipError_t e = launch_pcg_persistent(a, L.nv, cf, L.g, L.tab, max_blocks, cooperative, h->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    L.persistent = false;
    return false;
  }
  if (!h->capturing) porder_after(po, h, overlap);
  if (h->ptime) HIPCHECK(hipEventRecord(h->pev[2 * slot + 1], h->stream));
  h->ring_timed.push_back(h->ptime ? 1 : 0);
  h->ring_meta.emplace_back((int)(&L - h->lv.data()), maxit);
  h->ring_n += 1;
  conserve_fix(h, L, b, b ? nullptr : bl, x);
  return true;
}

// Multi-kernel Jacobi-PCG (Chronopoulos-Gear form) in precision T; x holds
// the initial guess on entry.  Iterations are enqueued in batches; the host
// reads the convergence record once per batch.  Returns the iterations, the
// The inverse Jacobi diagonal of an isotropic solve: from the level's cache
// when the level's own buffers serve the solve, else formed into B.idg.
template <typename T>
const T* iso_idg(sisdc_handle* h, Level& L, const CGBufs<T>& B, const CoefT<T>& cf, T dtm, T ctau) {
  constexpr bool f64 = std::is_same<T, double>::value;
  Level::IdgCache& C = f64 ? L.idgc64 : L.idgc32;
  if (!C.tab || (const void*)B.idg != (f64 ? (const void*)L.idg : (const void*)L.idg32)) {
    HIPCHECK(launch_iso_inv_diag(B.diag, B.idg, cf, dtm, ctau, L.g, B.tab, h->stream));
    return B.idg;
  }
  const double key[3] = {(double)dtm, (double)cf.nu, (double)ctau};
  T* const tab = (T*)C.tab;
  for (int k = 0; k < C.n; ++k)
    if (C.key[k][0] == key[0] && C.key[k][1] == key[1] && C.key[k][2] == key[2]) return tab + (long)k * L.np;
  const int k = C.n < Level::IdgCache::kSlots ? C.n++ : (C.next++ % Level::IdgCache::kSlots);
  for (int j = 0; j < 3; ++j) C.key[k][j] = key[j];
  HIPCHECK(launch_iso_inv_diag(B.diag, tab + (long)k * L.np, cf, dtm, ctau, L.g, B.tab, h->stream));
  return tab + (long)k * L.np;
}

// convergence flag and the final relative (recurred) residual.
template <typename T>
// b == NULL: the right-hand side is the combination bl (isotropic levels
// only: the start kernel forms it node by node).  x0 != NULL: the initial
// guess, when x does not hold it (on isotropic levels no copy to x is made;
// the first update of x reads x0).
sisdc_solve_stats cg_multi(sisdc_handle* h, Level& L, const CGBufs<T>& B, const CoefT<T>& cf, T dtm, const T* b, T* x,
                           double rtol, int maxit, bool x_is_zero, const LinComb* bl = nullptr,
                           const T* x0 = nullptr) {
  if (h->capturing) throw CaptureNeedsHost{};  // the host reads the convergence record
  hipStream_t s = h->stream;
  const int id = ++h->solve_id;
  const T ctau = (T)h->ctau, one = (T)1;
  // isotropic hexahedral levels: streaming CG, z = r / diag formed inside the matvec
  const bool iso = sipg_iso_path(L.g, cf);
  if (x0 == x || x_is_zero) x0 = nullptr;
  if (x0 && !iso) {
    copy_any(h, x, x0, L.vlen);
    x0 = nullptr;
  }
  if (!b && !(iso && bl)) fail(SISDC_EINVAL, "internal: no right-hand side for the multi-kernel PCG");
  CGStateT<T> cg = cg_state<T>(h, B, b, x, rtol);
  cg.x0 = x0;
  if (iso && B.cons && fused_conserve(h, L) && !x_is_zero) {  // the shift is fused into the PCG's kernels
    cg.cons = B.cons;
    cg.vs = L.vs;
    cg.nv = L.nv;
    cg.nparts = iso_cg_grid(L.g);
    cg.mass_total = (T)L.mass_total;
    if (L.nv > kMaxComp) fail(SISDC_EINVAL, "internal: more components than the conservation sums hold");
  }
  const T* const idg = iso ? iso_idg<T>(h, L, B, cf, dtm, ctau) : nullptr;
  if (!iso) HIPCHECK(launch_helm_diag(B.diag, L.nv, cf, dtm, ctau, L.g, B.tab, s));
  if (x_is_zero) {  // start from x = 0, so A x0 = 0
    HIPCHECK(hipMemsetAsync(x, 0, L.vlen * sizeof(T), s));
    HIPCHECK(hipMemsetAsync(B.w, 0, L.vlen * sizeof(T), s));
  } else {
    HIPCHECK(launch_sipg(x0 ? x0 : x, B.w, L.nv, cf, B.trace, one, dtm, ctau, L.g, B.tab, s));  // A x0
  }
  // element-block Jacobi by fast diagonalisation (FP64 isotropic levels): z
  // is stored; its kernel follows every update and replaces the update's
  // (r, z) and (r, r) partials, and the matvec reads z
  T* const zfds = (iso && h->meth.precond == SISDC_PRECOND_FDS && std::is_same<T, double>::value && L.fds)
                      ? B.z : nullptr;
  const double dtk = (double)dtm * (double)cf.nu;
  auto fds_step = [&](int k, const int* dg, int sid) {  // z = A_ee^-1 r, partials of iteration k
    HIPCHECK(launch_fds((const double*)B.r, (double*)zfds, L.nv, L.g, L.fds, dtk,
                        (double*)(cg.gam + (k % 3) * cg.cap), (double*)(cg.rr + (k % 2) * cg.cap), dg, sid, s));
  };
  cg.zs = zfds;
  if (iso) {
    HIPCHECK(launch_cg_start_iso(cg, idg, L.nv, L.g, b ? nullptr : bl, L.mw, s));
    if (zfds) fds_step(0, nullptr, 0);
    HIPCHECK(launch_sipg_apply_iso(zfds ? zfds : B.r, zfds ? nullptr : idg, B.w, L.nv, cf, one, dtm, ctau, L.g,
                                   B.tab, cg.del, (const int*)nullptr, 0, s));
  } else {
    HIPCHECK(launch_cg_start(cg, L.nv, cf, L.g, B.tab, s));
    HIPCHECK(launch_sipg_apply(B.z, B.w, L.nv, cf, B.trace, one, dtm, ctau, L.g, B.tab, B.z, cg.del,
                               (const int*)nullptr, 0, s));
  }
  int chunk = std::max(2, L.last_iters + 1);
  int it = 0;
  bool converged = false;
  const int li = (int)(&L - h->lv.data());
  const bool timed = h->ptime && (size_t)(2 * li + 1) < h->kt_us.size() && (h->kt_solves++ % h->kt_stride) == 0;
  while (true) {
    const int first = it;
    const int stop = std::min(maxit + 1, it + chunk);  // iteration kernel `it` checks the residual after it updates
    if (timed)
      while (h->mev.size() < (size_t)(3 * (stop - first))) {
        hipEvent_t ev = nullptr;
        HIPCHECK(hipEventCreate(&ev));
        h->mev.push_back(ev);
      }
    for (; it < stop; ++it) {
      hipEvent_t* ev = timed ? &h->mev[3 * (it - first)] : nullptr;
      if (timed) HIPCHECK(hipEventRecord(ev[0], s));
      if (iso)
        HIPCHECK(launch_cg_iter_iso(cg, idg, L.nv, L.g, it, id, s));
      else
        HIPCHECK(launch_cg_iter(cg, L.nv, cf, L.g, B.tab, it, id, s));
      if (timed) HIPCHECK(hipEventRecord(ev[1], s));
      if (it < maxit) {
        if (zfds) fds_step(it + 1, (const int*)B.done_gen, id);
        if (iso)
          HIPCHECK(launch_sipg_apply_iso(zfds ? zfds : B.r, zfds ? nullptr : idg, B.w, L.nv, cf, one, dtm, ctau,
                                         L.g, B.tab, cg.del, (const int*)B.done_gen, id, s));
        else
          HIPCHECK(launch_sipg_apply(B.z, B.w, L.nv, cf, B.trace, one, dtm, ctau, L.g, B.tab, B.z, cg.del,
                                     (const int*)B.done_gen, id, s));
      }
      if (timed) HIPCHECK(hipEventRecord(ev[2], s));
    }
    if ((const char*)B.done_gen == (const char*)B.res + kDoneOffset) {  // one copy for both
      HIPCHECK(hipMemcpyAsync(h->hres, B.res, kDoneOffset + sizeof(int), hipMemcpyDeviceToHost, s));
    } else {
      HIPCHECK(hipMemcpyAsync(h->hres, B.res, sizeof(CGRes), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipMemcpyAsync(h->hdone, B.done_gen, sizeof(int), hipMemcpyDeviceToHost, s));
    }
    HIPCHECK(hipStreamSynchronize(s));
    const bool done = *h->hdone == id;
    if (timed) {
      // launches before the converged iteration did a full iteration's work;
      // the converged one only tests, later ones exit at once
      const int full_end = done ? std::min(stop, h->hres->it) : stop;
      for (int k = first; k < full_end; ++k) {
        const hipEvent_t* ev = &h->mev[3 * (k - first)];
        float ms = 0.0f;
        HIPCHECK(hipEventElapsedTime(&ms, ev[0], ev[1]));
        h->kt_us[2 * li] += 1000.0 * ms;
        h->kt_n[2 * li] += 1;
        if (k < maxit) {
          HIPCHECK(hipEventElapsedTime(&ms, ev[1], ev[2]));
          h->kt_us[2 * li + 1] += 1000.0 * ms;
          h->kt_n[2 * li + 1] += 1;
        }
      }
    }
    if (done) {
      converged = true;
      break;
    }
    if (it > maxit) break;
    chunk = 8;
  }
  if (iso) HIPCHECK(launch_cg_fix_iso(cg, L.vlen, id, s));
  sisdc_solve_stats r{};
  r.iters = converged ? h->hres->it : maxit;
  const double rel = h->hres->bb > 0.0 ? std::sqrt(h->hres->rr / h->hres->bb) : 0.0;
  r.rel_residual = rel;
  r.converged = converged;
  if (!std::isfinite(rel) || !std::isfinite(h->hres->rr) || !std::isfinite(h->hres->bb))
    fail(SISDC_ENONFINITE, "non-finite residual in the Helmholtz solve");
  L.last_iters = std::max(1, r.iters);
  return r;
}

CoefT<float> coef32(sisdc_handle* h, Level& L, const CoefP& cf) {
  CoefT<float> c{};
  c.c = (float)cf.c;
  for (int d = 0; d < 3; ++d) c.v[d] = (float)cf.v[d];
  c.nu = (float)cf.nu;
  c.ub = nullptr;
  if (cf.ub) {
    HIPCHECK(launch_cast_f(cf.ub, L.ub32, L.vs, h->stream));  // the coefficient state is one scalar field
    c.ub = L.ub32;
  }
  return c;
}

// Mixed precision (FP64 iterative refinement around FP32 PCG):
//   r = b - A x (FP64); stop when ||r|| <= rtol ||b||; solve A e = r in FP32
//   to a relative tolerance max(inner_rtol, rtol ||b|| / (2 ||r||)); x += e.
sisdc_solve_stats mixed_solve(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, double* x,
                              double rtol, int maxit) {
  if (h->capturing) throw CaptureNeedsHost{};  // the host decides every refinement round
  hipStream_t s = h->stream;
  const CoefT<float> cf32 = coef32(h, L, cf);
  CGBufs<float> B = bufs32(h, L);
  sisdc_solve_stats out{};
  int total = 0, rounds = 0;
  double rel = 0.0, rel_prev = 0.0;
  bool converged = false, stalled = false;
  const double inner = h->meth.inner_rtol > 0.0 ? h->meth.inner_rtol : 1e-5;
  while (true) {
    HIPCHECK(launch_sipg(x, L.cw, L.nv, cf, L.trace, 1.0, dtm, h->ctau, L.g, L.tab, s));
    HIPCHECK(launch_resid_cast(b, L.cw, L.r32, L.vlen, h->partials, h->ir_tot, s));
    HIPCHECK(hipMemcpyAsync(h->hir_tot, h->ir_tot, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double rr = h->hir_tot[0], bb = h->hir_tot[1];
    rel = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    if (!std::isfinite(rel) || !std::isfinite(rr) || !std::isfinite(bb))
      fail(SISDC_ENONFINITE, "non-finite residual in the Helmholtz solve");
    if (rr <= rtol * rtol * bb) {
      converged = true;
      break;
    }
    if (total >= maxit) break;
    // refinement that no longer halves the FP64 residual per round (or runs
    // out of rounds) has stalled: FP64 PCG finishes the solve
    if (rounds >= 20 || (rounds > 0 && rel > 0.5 * rel_prev)) {
      stalled = true;
      break;
    }
    rel_prev = rel;
    const double tol_in = std::max(inner, 0.5 * rtol * std::sqrt(bb / rr));
    sisdc_solve_stats ri = cg_multi<float>(h, L, B, cf32, (float)dtm, L.r32, L.e32, tol_in, maxit - total, true);
    total += ri.iters;
    rounds += 1;
    HIPCHECK(launch_add_f2d(x, L.e32, L.vlen, s));
  }
  if (stalled) {
    sisdc_solve_stats r64 = cg_multi<double>(h, L, bufs64(h, L), cf, dtm, b, x, rtol, maxit - total, false);
    total += r64.iters;
    converged = r64.converged != 0;
    rel = r64.rel_residual;
    h->st.ir_fallbacks += 1;
  }
  out.iters = total;
  out.converged = converged;
  out.rel_residual = rel;
  h->st.ir_rounds += rounds;
  account(h, total, converged, rel);
  return out;
}

// ------------------------------------------------------------------ learned guess
// r = b - A x into out (FP64), with (r,r), (b,b) into tot[0..1] on the device
void residual64(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, const double* x, double* out,
                double* tot) {
  HIPCHECK(launch_sipg(x, L.cw, L.nv, cf, L.trace, 1.0, dtm, h->ctau, L.g, L.tab, h->stream));
  if (out) lincomb(h, L, out, {{1.0, b}, {-1.0, L.cw}});
  if (tot) {
    if (!L.r32) fail(SISDC_EDEVICE, "internal: FP32 staging missing");
    HIPCHECK(launch_resid_cast(b, L.cw, L.r32, L.vlen, h->partials, tot, h->stream));
  }
}

// The network proposes, for every (element, component) row, the correction
// delta_row = |z0_row| N(z0_row / |z0_row|), z0 = M^-1 (b - A x0); the guess
// moves along delta by the step that minimises the A-norm of the error,
// x0 <- x0 + alpha delta, alpha = (delta, r0) / (delta, A delta), so it can
// only lower that norm (a step that is not positive is refused; decided on
// the device).
void learned_guess(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, double* x) {
  auto& N = L.net;
  hipStream_t s = h->stream;
  const int rows = L.nv * L.E;
  residual64(h, L, cf, dtm, b, x, N.r0h, nullptr);
  HIPCHECK(launch_row_normalise(N.r0h, rows, L.np, L.mw, N.Xi, N.nrm, s));
  HIPCHECK(mlp_forward(N.sh, N.theta, N.Xi, rows, nullptr, N.A1i, nullptr, N.A2i, N.Yi, 1, s));
  HIPCHECK(launch_guess_delta(N.Yi, N.nrm, rows, L.np, N.xnew, s));
  HIPCHECK(launch_sipg(N.xnew, L.cw, L.nv, cf, L.trace, 1.0, dtm, h->ctau, L.g, L.tab, s));  // A delta
  HIPCHECK(launch_dot2(N.xnew, N.r0h, L.cw, L.vlen, h->partials, h->gtot, s));
  HIPCHECK(launch_guess_step(x, N.xnew, L.vlen, h->gtot, h->nrej, s));
  h->st.net_guesses += 1;
}

// record r0 = b - A x0 and x0 before a solve (harvest)
void harvest_before(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, const double* x) {
  auto& N = L.net;
  residual64(h, L, cf, dtm, b, x, N.r0h, nullptr);
  copy_d2d(h, N.x0h, x, L.vlen);
}

// append the rows (z0 / |z0|, (x* - x0) / |z0|), z0 = M^-1 r0, of the finished solve
void harvest_after(sisdc_handle* h, Level& L, const double* x) {
  auto& N = L.net;
  const int rows = L.nv * L.E;
  if (N.rows + rows > N.max_rows) return;
  HIPCHECK(launch_row_normalise(N.r0h, rows, L.np, L.mw, N.Xi, N.nrm, h->stream));
  HIPCHECK(launch_harvest(N.r0h, x, N.x0h, N.nrm, rows, L.np, L.mw, N.Xd + (long)N.rows * L.np,
                          N.Td + (long)N.rows * L.np, h->stream));
  N.rows += rows;
}

sisdc_solve_stats cg_solve_core(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, double* x,
                                double rtol, int maxit);

sisdc_solve_stats cg_solve(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, double* x,
                           double rtol, int maxit) {
  const bool harvest = L.net.on && L.net.harvest && L.net.rows < L.net.max_rows;
  if (harvest) harvest_before(h, L, cf, dtm, b, x);
  if (L.net.on && L.net.use) learned_guess(h, L, cf, dtm, b, x);
  sisdc_solve_stats r = cg_solve_core(h, L, cf, dtm, b, x, rtol, maxit);
  if (harvest) harvest_after(h, L, x);
  return r;
}

sisdc_solve_stats cg_solve_core(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, double* x,
                                double rtol, int maxit) {
  if (h->meth.precision == SISDC_MIXED) {
    sisdc_solve_stats r = mixed_solve(h, L, cf, dtm, b, x, rtol, maxit);
    conserve_fix(h, L, b, nullptr, x);
    return r;
  }
  // the pipelined persistent form is used for production tolerances only
  if (L.persistent && rtol >= kPersistentMinRtol && persistent_solve(h, L, cf, dtm, b, x, rtol, maxit)) {
    sisdc_solve_stats r{};
    r.iters = -1;  // collected later by drain()
    r.converged = 1;
    return r;
  }
  sisdc_solve_stats r = cg_multi<double>(h, L, bufs64(h, L), cf, dtm, b, x, rtol, maxit, false);
  account(h, r.iters, r.converged, r.rel_residual);
  if (!(sipg_iso_path(L.g, cf) && fused_conserve(h, L))) conserve_fix(h, L, b, nullptr, x);
  return r;
}

// Plain FP64 solves on isotropic levels (the systems' kappa_m I) run the
// streaming multi-kernel PCG straight from the right-hand side's combination
// (formed node by node in its start kernel) and from x0 (read by its first
// update of x): no assembly pass and no copy of x0.
bool stream_iso(sisdc_handle* h, const Level& L, const CoefP& cf) {
  return h->meth.precision == SISDC_FP64 && sipg_iso_path(L.g, cf);
}

sisdc_solve_stats solve_iso(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b,
                            const LinComb* bl, double* x, const double* x0) {
  sisdc_solve_stats r = cg_multi<double>(h, L, bufs64(h, L), cf, dtm, b, x, h->meth.cg_rtol, h->meth.cg_maxit, false,
                                         bl, x0);
  account(h, r.iters, r.converged, r.rel_residual);
  if (!fused_conserve(h, L)) conserve_fix(h, L, b, b ? nullptr : bl, x);
  return r;
}

// Solve with the initial guess x0 (x0 == x: x holds it).  The persistent
// PCG reads x0 and writes x itself; the other forms start from a copy.
sisdc_solve_stats solve(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const double* b, double* x,
                        const double* x0) {
  const double rtol = h->meth.cg_rtol;
  const bool plain = !(L.net.on && (L.net.use || L.net.harvest)) && h->meth.precision != SISDC_MIXED;
  if (x0 != x && plain && L.persistent && rtol >= kPersistentMinRtol &&
      persistent_solve(h, L, cf, dtm, b, x, rtol, h->meth.cg_maxit, x0)) {
    sisdc_solve_stats r{};
    r.iters = -1;  // collected later by drain()
    r.converged = 1;
    return r;
  }
  if (x0 != x && plain && stream_iso(h, L, cf)) return solve_iso(h, L, cf, dtm, b, nullptr, x, x0);
  if (x0 != x) copy_d2d(h, x, x0, L.vlen);
  return cg_solve(h, L, cf, dtm, b, x, rtol, h->meth.cg_maxit);
}

// Solve with the right-hand side given as a combination of vectors: the
// persistent PCG forms it at every node itself (no separate assembly
// kernel); the other forms get it assembled into L.b first.
sisdc_solve_stats solve_lc(sisdc_handle* h, Level& L, const CoefP& cf, double dtm, const LinComb& lc, double* x,
                           const double* x0) {
  const double rtol = h->meth.cg_rtol;
  const bool plain = !(L.net.on && (L.net.use || L.net.harvest)) && h->meth.precision != SISDC_MIXED;
  if (plain && L.persistent && rtol >= kPersistentMinRtol &&
      persistent_solve(h, L, cf, dtm, nullptr, x, rtol, h->meth.cg_maxit, x0, &lc)) {
    sisdc_solve_stats r{};
    r.iters = -1;  // collected later by drain()
    r.converged = 1;
    return r;
  }
  if (plain && stream_iso(h, L, cf)) return solve_iso(h, L, cf, dtm, nullptr, &lc, x, x0);
  HIPCHECK(launch_lincomb(L.b, lc, L.vlen, L.mw, L.np, h->stream));
  return solve(h, L, cf, dtm, L.b, x, x0);
}

// ------------------------------------------------------------------ sweeps
// Stored terms of the current iterate: C(u_m), m = 0..M; f(u_m) and
// X_m = K_{D_m(u_{m-1})} u_m, m = 1..M (implementation note of Sec. 3:
// the f of sweep k-1 are kept).
void ensure_stored(sisdc_handle* h, Level& L, double dt) {
  if (!L.stale && L.stored_dt == dt) return;
  conv(h, L, L.um(0), L.C, L.M + 1);  // all nodes in one launch (node vectors are consecutive)
  // f_m = C_m - K_nu u_m of all nodes in one launch where the isotropic kernel
  // applies: the M node vectors act as M nv independent components
  const bool f_batched = has_physical_diffusion(h) && L.g.dim == 2 &&
                         launch_sipg_iso2_add(L.um(1), L.C + L.vlen, L.f, L.nv * L.M, coef_nu(h), 0.0, -1.0, h->ctau,
                                              L.g, L.tab, h->stream) == hipSuccess;
  if (!f_batched) (void)hipGetLastError();
  for (int m = 1; m <= L.M; ++m) {
    const double dtm = dt * L.dtau[m - 1];
    if (!f_batched) frhs_from_c(h, L, L.um(m), L.C + (long)m * L.vlen, L.f + (long)(m - 1) * L.vlen);
    sipg(h, L, coef_for(h, L, dtm, L.um(m - 1)), L.um(m), L.X + (long)(m - 1) * L.vlen, 0.0, 1.0);
  }
  L.stale = false;
  L.stored_dt = dt;
}

// q_m = sum_i S_{m,i} f_i, S = dt w^nn, for m = 1..M (one pass over the f_i)
void quadrature(sisdc_handle* h, Level& L, double dt) {
  if (L.M <= 8) {
    LinCombMulti lc{};
    lc.nin = L.M;
    lc.nout = L.M;
    for (int i = 0; i < L.M; ++i) lc.x[i] = L.f + (long)i * L.vlen;
    for (int m = 0; m < L.M; ++m)
      for (int i = 0; i < L.M; ++i) lc.c[m][i] = dt * L.wnn[m * L.M + i];
    HIPCHECK(launch_lincomb_multi(L.q, lc, L.vlen, h->stream));
    return;
  }
  for (int m = 0; m < L.M; ++m) {
    std::vector<double> c;
    std::vector<const double*> x;
    for (int i = 0; i < L.M; ++i) {
      c.push_back(dt * L.wnn[m * L.M + i]);
      x.push_back(L.f + (long)i * L.vlen);
    }
    lincomb_v(h, L, L.q + (long)m * L.vlen, c, x, {});
  }
}

void predictor(sisdc_handle* h, Level& L, double dt) {
  const bool si1 = h->meth.integrator != SISDC_SI2;  // one-stage forms: SI(1), IMEX Euler
  for (int m = 1; m <= L.M; ++m) {
    const double dtm = dt * L.dtau[m - 1];
    const double* ua = L.um(m - 1);
    CoefP cf = coef_for(h, L, dtm, ua);
    conv(h, L, ua, L.t1);
    double* y = si1 ? L.um(m) : L.y;
    solve_lc(h, L, cf, dtm, make_lc({{1.0, ua}, {dtm, L.t1}}, {1, 0}), y, ua);
    if (!si1) {
      conv(h, L, y, L.t1);
      solve_lc(h, L, cf, dtm, make_lc({{1.0, ua}, {dtm, L.t1}}, {1, 0}), L.um(m), y);
    }
  }
  L.stale = true;
}

// One incremental SI(1)/SI(2) corrector sweep (Alg. 1 with N = 1).
void sweep(sisdc_handle* h, Level& L, double dt, const double* g) {
  const bool si1 = h->meth.integrator != SISDC_SI2;  // one-stage forms: SI(1), IMEX Euler
  ensure_stored(h, L, dt);
  quadrature(h, L, dt);
  const long n = L.vlen;
  copy_d2d(h, L.unm(0), L.um(0), n);
  copy_d2d(h, L.Cnew, L.C, n);
  for (int m = 1; m <= L.M; ++m) {
    const double dtm = dt * L.dtau[m - 1];
    const double* ua = L.unm(m - 1);
    const double* Ca = L.Cnew + (long)(m - 1) * n;
    const double* qm = L.q + (long)(m - 1) * n;
    const double* Xm = L.X + (long)(m - 1) * n;
    const double* Cold_prev = L.C + (long)(m - 1) * n;
    const double* Cold_m = L.C + (long)m * n;
    const double* gm = g ? g + (long)(m - 1) * n : nullptr;
    CoefP cf = coef_for(h, L, dtm, ua);
    // stage 1: M y = M u^k_{m-1} + q_m + g_m + H(u^k_{m-1},u^k_{m-1},y) - H(u^{k-1}_{m-1},u^{k-1}_{m-1},u^{k-1}_m)
    const LinComb b1 =
        gm ? make_lc({{1.0, ua}, {1.0, qm}, {1.0, gm}, {dtm, Ca}, {-dtm, Cold_prev}, {dtm, Xm}}, {1, 0, 0, 0, 0, 0})
           : make_lc({{1.0, ua}, {1.0, qm}, {dtm, Ca}, {-dtm, Cold_prev}, {dtm, Xm}}, {1, 0, 0, 0, 0});
    double* y = si1 ? L.unm(m) : L.y;
    // initial guess: u^{k-1}_m shifted by the change this sweep made at node
    // m-1 (the corrections of neighbouring nodes are close); the guess moves
    // the PCG iterates only, not the solution it converges to
    const double* x0 = L.um(m);
    if (m > 1) {
      lincomb(h, L, L.t2, {{1.0, L.um(m)}, {1.0, L.unm(m - 1)}, {-1.0, L.um(m - 1)}});
      x0 = L.t2;
    }
    solve_lc(h, L, cf, dtm, b1, y, x0);
    if (!si1) {
      // stage 2: M u^k_m = M u^k_{m-1} + q_m + g_m + H(y,u^k_{m-1},u^k_m) - H(u^{k-1}_m,u^{k-1}_{m-1},u^{k-1}_m)
      conv(h, L, y, L.t1);
      const LinComb b2 =
          gm ? make_lc({{1.0, ua}, {1.0, qm}, {1.0, gm}, {dtm, L.t1}, {-dtm, Cold_m}, {dtm, Xm}}, {1, 0, 0, 0, 0, 0})
             : make_lc({{1.0, ua}, {1.0, qm}, {dtm, L.t1}, {-dtm, Cold_m}, {dtm, Xm}}, {1, 0, 0, 0, 0});
      solve_lc(h, L, cf, dtm, b2, L.unm(m), y);
    }
    // stored terms of the new iterate at node m
    double* Cm = L.Cnew + (long)m * n;
    conv(h, L, L.unm(m), Cm);
    sipg(h, L, cf, L.unm(m), L.X + (long)(m - 1) * n, 0.0, 1.0);
    frhs_from_c(h, L, L.unm(m), Cm, L.f + (long)(m - 1) * n);
  }
  std::swap(L.u, L.unew);
  std::swap(L.C, L.Cnew);
  L.stale = false;
  L.stored_dt = dt;
}

// F_m(u) = M (u_m - u_{m-1}) - q_m(u) into out[m-1]; with g_minus, g_m - F_m(u);
// with negate (and no g_minus), -F_m(u)
void colloc_residual(sisdc_handle* h, Level& L, double dt, double* out, const double* g_minus,
                     bool negate = false) {
  ensure_stored(h, L, dt);
  if (L.M <= 8) {
    CollocResid c{};
    c.u = L.u;
    c.f = L.f;
    c.g = g_minus;
    c.out = out;
    c.M = L.M;
    c.sign = (g_minus || negate) ? -1.0 : 1.0;
    for (int m = 0; m < L.M; ++m)
      for (int i = 0; i < L.M; ++i) c.S[m][i] = dt * L.wnn[m * L.M + i];
    HIPCHECK(launch_colloc_residual(c, L.vlen, L.mw, L.np, h->stream));
    return;
  }
  quadrature(h, L, dt);
  for (int m = 1; m <= L.M; ++m) {
    double* o = out + (long)(m - 1) * L.vlen;
    const double* qm = L.q + (long)(m - 1) * L.vlen;
    if (g_minus)  // r = g - F
      lincomb(h, L, o, {{1.0, g_minus + (long)(m - 1) * L.vlen}, {-1.0, L.um(m)}, {1.0, L.um(m - 1)}, {1.0, qm}},
              {0, 1, 1, 0});
    else if (negate)
      lincomb(h, L, o, {{-1.0, L.um(m)}, {1.0, L.um(m - 1)}, {1.0, qm}}, {1, 1, 0});
    else
      lincomb(h, L, o, {{1.0, L.um(m)}, {-1.0, L.um(m - 1)}, {-1.0, qm}}, {1, 1, 0});
  }
}

void space_transfer(sisdc_handle* h, const Level& from, const Level& to, const double* in, double* out,
                    const double* A) {
  if (from.E == to.E) {
    HIPCHECK(launch_space_transfer(in, out, from.nv, from.g.dim, from.n1, to.n1, from.E, A, h->stream));
    return;
  }
  const int dim = from.g.dim;
  if (from.E == (to.E << dim)) {  // fine -> coarse over 2:1 h-coarsening
    HIPCHECK(launch_space_transfer_h(in, out, from.nv, dim, from.n1, to.n1, to.g.ne, A, 0, h->stream));
  } else if (to.E == (from.E << dim)) {  // coarse -> fine
    HIPCHECK(launch_space_transfer_h(in, out, from.nv, dim, to.n1, from.n1, from.g.ne, A, 1, h->stream));
  } else {
    fail(SISDC_EINVAL, "internal: levels are not related by 2:1 h-coarsening");
  }
}

// Space-time transfer in one launch between levels with the same elements
// (the callers check st_fits and the element counts first, and otherwise
// transfer node by node).
void st_transfer(sisdc_handle* h, const Level& from, const Level& to, const TransferMulti& t, const double* A) {
  if (from.E != to.E) fail(SISDC_EINVAL, "internal: one-launch transfer between different meshes");
  HIPCHECK(launch_space_time_transfer(t, from.nv, from.g.dim, from.n1, to.n1, from.E, A, h->stream));
}

bool st_fits(int nin, int nout) { return nin <= kTransferIn && nout <= kTransferOut; }

// FAS restriction from fine level i to coarse level i+1 (Alg. 2, residual
// evaluation, solution restriction and RHS composition).
void restrict_fas(sisdc_handle* h, int i, double dt) {
  Level& F = h->lv[i];
  Level& Cc = h->lv[i + 1];
  Transfer& T = h->tr[i];
  colloc_residual(h, F, dt, F.r, F.has_g ? F.gf : nullptr, true);  // r = g - F(u), g = 0 on the top level
  // v_c = (P_t x P_x) u_f, v_c[0] = coarse u_0; u_c <- v_c
  copy_d2d(h, Cc.v, Cc.um(0), Cc.vlen);
  const bool one_launch = F.E == Cc.E && st_fits(F.M, Cc.M);
  if (one_launch) {
    TransferMulti t{};
    t.nin = F.M;
    t.nout = Cc.M;
    for (int j = 0; j < F.M; ++j) t.x[j] = F.um(j + 1);
    for (int mc = 0; mc < Cc.M; ++mc) {
      for (int j = 0; j < F.M; ++j) t.c[mc][j] = T.Pt[mc * F.M + j];
      t.y[mc] = Cc.v + (long)(mc + 1) * Cc.vlen;
      t.y2[mc] = Cc.um(mc + 1);
    }
    st_transfer(h, F, Cc, t, T.Px);
  } else {
    for (int mc = 0; mc < Cc.M; ++mc) {
      std::vector<double> c;
      std::vector<const double*> x;
      for (int j = 0; j < F.M; ++j) {
        c.push_back(T.Pt[mc * F.M + j]);
        x.push_back(F.um(j + 1));
      }
      lincomb_v(h, F, F.t1, c, x, {});
      space_transfer(h, F, Cc, F.t1, Cc.v + (long)(mc + 1) * Cc.vlen, T.Px);
    }
    copy_d2d(h, Cc.u, Cc.v, (long)(Cc.M + 1) * Cc.vlen);
  }
  // g_c = F_c(v_c) + R r_f
  Cc.stale = true;
  Cc.has_g = false;
  colloc_residual(h, Cc, dt, Cc.gf, nullptr);
  if (one_launch) {
    TransferMulti t{};
    t.nin = F.M;
    t.nout = Cc.M;
    t.accumulate = 1;
    for (int i2 = 0; i2 < F.M; ++i2) t.x[i2] = F.r + (long)i2 * F.vlen;
    for (int mc = 0; mc < Cc.M; ++mc) {
      for (int i2 = 0; i2 < F.M; ++i2) t.c[mc][i2] = T.Rt[mc * F.M + i2];
      t.y[mc] = Cc.gf + (long)mc * Cc.vlen;
    }
    st_transfer(h, F, Cc, t, T.Rx);
  } else {
    for (int mc = 0; mc < Cc.M; ++mc) {
      std::vector<double> c;
      std::vector<const double*> x;
      for (int i2 = 0; i2 < F.M; ++i2) {
        c.push_back(T.Rt[mc * F.M + i2]);
        x.push_back(F.r + (long)i2 * F.vlen);
      }
      lincomb_v(h, F, F.t1, c, x, {});
      space_transfer(h, F, Cc, F.t1, Cc.t1, T.Rx);
      double* gm = Cc.gf + (long)mc * Cc.vlen;
      lincomb(h, Cc, gm, {{1.0, gm}, {1.0, Cc.t1}});
    }
  }
  Cc.has_g = true;
}

// u_f[m] += (I_t x I_x)(u_c - v_c)[m], m = 1..M_f (correction prolongation)
void prolong_correction(sisdc_handle* h, int i) {
  Level& F = h->lv[i];
  Level& Cc = h->lv[i + 1];
  Transfer& T = h->tr[i];
  if (F.E == Cc.E && st_fits(2 * Cc.M, F.M)) {
    TransferMulti t{};
    t.nin = 2 * Cc.M;
    t.nout = F.M;
    t.accumulate = 1;
    for (int j = 0; j < Cc.M; ++j) {
      t.x[2 * j] = Cc.um(j + 1);
      t.x[2 * j + 1] = Cc.v + (long)(j + 1) * Cc.vlen;
    }
    for (int mf = 0; mf < F.M; ++mf) {
      for (int j = 0; j < Cc.M; ++j) {
        t.c[mf][2 * j] = T.It[mf * Cc.M + j];
        t.c[mf][2 * j + 1] = -T.It[mf * Cc.M + j];
      }
      t.y[mf] = F.um(mf + 1);
    }
    st_transfer(h, Cc, F, t, T.Ix);
    F.stale = true;
    return;
  }
  for (int mf = 0; mf < F.M; ++mf) {
    std::vector<double> c;
    std::vector<const double*> x;
    for (int j = 0; j < Cc.M; ++j) {
      c.push_back(T.It[mf * Cc.M + j]);
      x.push_back(Cc.um(j + 1));
      c.push_back(-T.It[mf * Cc.M + j]);
      x.push_back(Cc.v + (long)(j + 1) * Cc.vlen);
    }
    lincomb_v(h, Cc, Cc.t1, c, x, {});
    space_transfer(h, Cc, F, Cc.t1, F.t1, T.Ix);
    lincomb(h, F, F.um(mf + 1), {{1.0, F.um(mf + 1)}, {1.0, F.t1}});
  }
  F.stale = true;
}

// u_f[m] = (I_t x I_x) u_c [m], m = 1..M_f  (cascade / FMG interpolation)
void interpolate_up(sisdc_handle* h, int i) {
  Level& F = h->lv[i];
  Level& Cc = h->lv[i + 1];
  Transfer& T = h->tr[i];
  if (F.E == Cc.E && st_fits(Cc.M, F.M)) {
    TransferMulti t{};
    t.nin = Cc.M;
    t.nout = F.M;
    for (int j = 0; j < Cc.M; ++j) t.x[j] = Cc.um(j + 1);
    for (int mf = 0; mf < F.M; ++mf) {
      for (int j = 0; j < Cc.M; ++j) t.c[mf][j] = T.It[mf * Cc.M + j];
      t.y[mf] = F.um(mf + 1);
    }
    st_transfer(h, Cc, F, t, T.Ix);
    F.stale = true;
    return;
  }
  for (int mf = 0; mf < F.M; ++mf) {
    std::vector<double> c;
    std::vector<const double*> x;
    for (int j = 0; j < Cc.M; ++j) {
      c.push_back(T.It[mf * Cc.M + j]);
      x.push_back(Cc.um(j + 1));
    }
    lincomb_v(h, Cc, Cc.t1, c, x, {});
    space_transfer(h, Cc, F, Cc.t1, F.um(mf + 1), T.Ix);
  }
  F.stale = true;
}

void level_sweep(sisdc_handle* h, int i, double dt) {
  Level& L = h->lv[i];
  sweep(h, L, dt, L.has_g ? L.gf : nullptr);
  if (i == 0) h->st.fine_sweeps += 1;
}

// Alg. 2 on levels top (finest of the cycle) .. coarsest; g = 0 on top.
void vcycle(sisdc_handle* h, int top, double dt) {
  const int Lc = (int)h->lv.size() - 1;
  h->lv[top].has_g = false;
  for (int i = top; i < Lc; ++i) {
    level_sweep(h, i, dt);
    restrict_fas(h, i, dt);
  }
  for (int k = 0; k < h->meth.n_coarse_sweeps; ++k) level_sweep(h, Lc, dt);
  for (int i = Lc - 1; i >= top; --i) {
    prolong_correction(h, i);
    if (i > top) level_sweep(h, i, dt);
  }
}

void set_level_initial(sisdc_handle* h) {
  copy_d2d(h, h->lv[0].um(0), h->state, h->lv[0].vlen);
  for (size_t i = 1; i < h->lv.size(); ++i)
    space_transfer(h, h->lv[i - 1], h->lv[i], h->lv[i - 1].um(0), h->lv[i].um(0), h->tr[i - 1].Px);
  for (auto& L : h->lv) {
    L.stale = true;
    L.has_g = false;
  }
}

// eps_e of the artificial viscosity from the fine-level state u.
void av_update(sisdc_handle* h, const double* u) {
  const Level& F = h->lv[0];
  HIPCHECK(launch_av_sensor(u, F.nv, F.g, h->eq, h->av_tab, h->meth.av_kappa, h->meth.av_c, h->eps, h->stream));
}

void update_lam(sisdc_handle* h) {
  if (!is_system(h)) {
    h->lam = 0.0;
    h->visc = 0.0;
    return;
  }
  if (h->capturing) throw CaptureNeedsHost{};  // the bound is read on the host
  Level& L = h->lv[0];
  HIPCHECK(launch_euler_lam(L.um(0), L.vs, h->eq, L.g.dim, h->partials, h->lam_dev, h->stream));
  HIPCHECK(hipMemcpyAsync(h->hlam, h->lam_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  h->lam = h->hlam[0];
  h->visc = 0.0;
  if (h->eq.eq == EQ_NS) {
    const double rmin = h->hlam[1];
    if (!(rmin > 0.0)) fail(SISDC_ENONFINITE, "non-positive density in the state");
    h->visc = std::max(4.0 * h->eq.mu / (3.0 * rmin), h->eq.gamma * h->eq.mu / (h->prob.Pr * rmin));
  }
}

// One time step up to the copy of the new state (everything but collecting
// the solves' records): the work a step graph captures.
void step_body(sisdc_handle* h, double dt) {
  set_level_initial(h);
  if (h->av) av_update(h, h->lv[0].um(0));
  update_lam(h);
  const int nl = (int)h->lv.size();
  const int Lc = nl - 1;
  if (nl == 1) {
    predictor(h, h->lv[0], dt);
    h->st.fine_sweeps += 1;
    for (int k = 0; k < h->meth.n_iter; ++k) level_sweep(h, 0, dt);
  } else {
    const int start = h->meth.start;
    if (start == SISDC_START_PREDICTOR) {
      for (int i = 0; i < nl; ++i) predictor(h, h->lv[i], dt);
      h->st.fine_sweeps += 1;
    } else if (start == SISDC_START_CONSTANT) {  // u_{l,m} = u_{l,0} on every node of every level
      for (auto& L : h->lv) {
        for (int m = 1; m <= L.M; ++m) copy_d2d(h, L.um(m), L.um(0), L.vlen);
        L.stale = true;
      }
    } else {
      predictor(h, h->lv[Lc], dt);
      if (start == SISDC_START_CASCADE) {  // Alg. 3
        for (int i = Lc; i >= 1; --i) {
          level_sweep(h, i, dt);
          interpolate_up(h, i - 1);
        }
      } else {  // Alg. 4: C_fmg V-cycles per added level
        const int cfmg = std::max(1, h->meth.c_fmg);
        level_sweep(h, Lc, dt);
        interpolate_up(h, Lc - 1);
        for (int i = Lc - 1; i >= 1; --i) {
          for (int c = 0; c < cfmg; ++c) vcycle(h, i, dt);
          interpolate_up(h, i - 1);
        }
      }
    }
    for (int c = 0; c < h->meth.n_iter; ++c) vcycle(h, 0, dt);
    if (h->meth.post_sweep) {
      h->lv[0].has_g = false;
      level_sweep(h, 0, dt);
    }
  }
  Level& F = h->lv[0];
  copy_d2d(h, h->state, F.um(F.M), F.vlen);
}

void do_step(sisdc_handle* h, double dt) {
  step_body(h, dt);
  drain(h);
  HIPCHECK(hipStreamSynchronize(h->stream));
}

// ------------------------------------------------------------------ step graphs
// A step whose every Helmholtz solve is a persistent PCG launch needs the host
// only at its end (to collect the solves' result records), so it can be
// captured once into a HIP graph and replayed: one launch per step instead of
// one per kernel.  Each solve still ends on its own convergence test on the
// device.  The graph bakes in the step size, the device buffers and the
// solver form; another dt or form captures again.  The persistent PCG's
// tagged records (barrier and face words) are cleared by the graph's first
// kernels and its tags restart from the captured values, so replays never
// meet stale tags.

// Why this handle's step cannot be captured (nullptr: it may be).
const char* graph_refusal(const sisdc_handle* h) {
  if (is_system(h)) return "the step's wave-speed bound is read on the host";
  if (h->meth.precision != SISDC_FP64) return "mixed-precision refinement is decided on the host";
  if (h->meth.cg_variant == SISDC_CG_PERSISTENT_COOPERATIVE) return "cooperative launches are not captured";
  if (h->meth.cg_rtol < kPersistentMinRtol) return "the tolerance takes the multi-kernel PCG";
  if (h->ptime) return "PCG event timing is on";
  for (const auto& L : h->lv) {
    if (!L.persistent) return "a level takes the multi-kernel PCG";
    if (L.net.on) return "a learned initial guess is in use";
  }
  return nullptr;
}

int graph_form(const sisdc_handle* h) { return h->meth.cg_variant * 8 + h->meth.precision; }

void graph_drop(sisdc_handle* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  h->gexec = nullptr;
}

// Capture one step (nothing runs).  False when the step needed the host.
bool capture_step(sisdc_handle* h, double dt) {
  graph_drop(h);
  drain(h);
  const unsigned tag_before = h->tag;
  const sisdc_stats saved = h->st;
  if (!h->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  hipStream_t const own = h->stream;
  auto reset = [&]() {
    h->stream = own;
    h->capturing = false;
    h->ring_n = 0;
    h->ring_meta.clear();
    h->ring_timed.clear();
    h->st = saved;
  };
  h->st = sisdc_stats{};
  h->tag = 0;
  // captured on a stream of its own (nothing runs there); the graph is
  // launched on the handle's stream
  HIPCHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
  h->stream = h->cap_stream;
  h->capturing = true;
  bool needs_host = false;
  try {
    clear_tagged_records(h);
    step_body(h, dt);
  } catch (const CaptureNeedsHost&) {
    needs_host = true;
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(h->cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    reset();
    h->tag = tag_before;
    throw;
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  const std::vector<std::pair<int, int>> meta = h->ring_meta;
  const sisdc_stats counted = h->st;
  reset();
  if (needs_host || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    h->tag = tag_before;  // nothing ran: the records still hold the earlier tags
    if (!needs_host) HIPCHECK(e);
    return false;
  }
  const hipError_t ei = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    h->gexec = nullptr;
    h->tag = tag_before;
    HIPCHECK(ei);
  }
  h->g_ring_meta = meta;
  h->g_st = counted;
  h->g_captures += 1;
  return true;
}

// Run one step through the handle's graph (capturing it first when needed).
// False, with nothing run, when the step cannot be captured.
bool graph_step(sisdc_handle* h, double dt) {
  if (graph_refusal(h)) {
    graph_drop(h);
    return false;
  }
  const int form = graph_form(h);
  if (h->g_refused_form == form && h->g_refused_dt == dt) return false;
  if (!h->gexec || h->g_dt != dt || h->g_form != form) {
    if (!capture_step(h, dt)) {
      h->g_refused_form = form;
      h->g_refused_dt = dt;
      return false;
    }
    h->g_dt = dt;
    h->g_form = form;
  }
  // the graph is ordered against other streams' persistent launches as one
  // launch: it may overlap other lanes when every level's grid may
  bool overlap = h->lane >= 0;
  for (const auto& L : h->lv) overlap = overlap && lane_may_overlap(h, L);
  PersistentOrder& po = porder(h->dev);
  {
    std::lock_guard<std::mutex> lock(po.m);
    porder_before(po, h, overlap);
    HIPCHECK(hipGraphLaunch(h->gexec, h->stream));
    porder_after(po, h, overlap);
  }
  h->g_replays += 1;
  h->st = h->g_st;
  h->ring_n = (int)h->g_ring_meta.size();
  h->ring_meta = h->g_ring_meta;
  h->ring_timed.assign(h->ring_n, 0);
  drain(h);
  HIPCHECK(hipStreamSynchronize(h->stream));
  return true;
}

// ------------------------------------------------------------------ setup
void build_level(sisdc_handle* h, Level& L, int P, int M, const int* ne) {
  const sisdc_problem& pr = h->prob;
  L.P = P;
  L.M = M;
  L.n1 = P + 1;
  L.np = pr.dim == 2 ? L.n1 * L.n1 : L.n1 * L.n1 * L.n1;
  L.E = 1;
  for (int d = 0; d < pr.dim; ++d) L.E *= ne[d];
  L.nv = h->eq.nv;
  L.vs = (long)L.E * L.np;
  L.vlen = L.vs * L.nv;
  Geo& g = L.g;
  g.dim = pr.dim;
  g.P = P;
  g.n1 = L.n1;
  g.np = L.np;
  g.nf = pr.dim == 2 ? L.n1 : L.n1 * L.n1;
  g.E = L.E;
  g.J = 1.0;
  const int stack = pr.stack > 1 ? pr.stack : 1;  // instances stacked along the last axis
  for (int d = 0; d < 3; ++d) {
    g.ne[d] = d < pr.dim ? ne[d] : 1;
    g.h[d] = d < pr.dim ? (pr.hi[d] - pr.lo[d]) / (d == pr.dim - 1 ? ne[d] / stack : ne[d]) : 1.0;
    g.rh2[d] = 2.0 / g.h[d];
    if (d < pr.dim) g.J *= 0.5 * g.h[d];
  }
  g.wl = g.ne[pr.dim - 1] / stack;
  gll(P, L.xg, L.wg);
  if ((int)L.xg.size() != L.n1) fail(SISDC_EDEVICE, "GLL node construction failed");
  L.D = derivative_matrix(L.xg);
  if (h->meth.nodes == SISDC_NODES_LOBATTO) {  // the M Gauss-Lobatto points mapped to [0, 1]
    std::vector<double> x, w;
    gll(M - 1, x, w);
    L.tau.assign(M, 0.0);
    for (int m = 0; m < M && m < (int)x.size(); ++m) L.tau[m] = 0.5 * (x[m] + 1.0);
    L.tau[0] = 0.0;
    L.tau[M - 1] = 1.0;
    if ((int)x.size() != M) fail(SISDC_EDEVICE, "Lobatto node construction failed");
  } else {
    L.tau = radau_right(M);
  }
  if ((int)L.tau.size() != M) fail(SISDC_EDEVICE, "collocation node construction failed");
  L.dtau.resize(M);
  for (int m = 0; m < M; ++m) L.dtau[m] = L.tau[m] - (m ? L.tau[m - 1] : 0.0);
  L.wnn = nn_weights(L.tau);
  std::vector<double> tab(L.D);
  tab.insert(tab.end(), L.wg.begin(), L.wg.end());
  L.tab = dalloc(tab.size());
  HIPCHECK(hipMemcpy(L.tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
  std::vector<double> mw(L.np);
  for (int n = 0; n < L.np; ++n) {
    int i0 = n % L.n1, i1 = (n / L.n1) % L.n1, i2 = n / (L.n1 * L.n1);
    double w = L.wg[i0] * L.wg[i1];
    if (pr.dim == 3) w *= L.wg[i2];
    mw[n] = g.J * w;
  }
  L.mw = dalloc(L.np);
  HIPCHECK(hipMemcpy(L.mw, mw.data(), L.np * sizeof(double), hipMemcpyHostToDevice));
  L.mass_total = 0.0;
  for (int n = 0; n < L.np; ++n) L.mass_total += mw[n];
  L.mass_total *= L.E;
  {  // fast diagonalisation of the isotropic element block, per axis (unit diffusivity)
    std::vector<double> ft((size_t)3 * L.n1 * L.n1 + 3 * L.n1, 0.0);
    for (int d = 0; d < 3; ++d) {
      std::vector<double> S, lam;
      if (d < pr.dim) {
        fds_axis(L.wg, L.D, g.rh2[d], h->ctau * (double)(L.n1 * L.n1), S, lam);
      } else {
        S.assign((size_t)L.n1 * L.n1, 0.0);
        for (int i = 0; i < L.n1; ++i) S[i * L.n1 + i] = 1.0;
        lam.assign(L.n1, 0.0);
      }
      std::copy(S.begin(), S.end(), ft.begin() + (size_t)d * L.n1 * L.n1);
      std::copy(lam.begin(), lam.end(), ft.begin() + (size_t)3 * L.n1 * L.n1 + d * L.n1);
    }
    L.fds = dalloc(ft.size());
    HIPCHECK(hipMemcpy(L.fds, ft.data(), ft.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  const long n = L.vlen;
  L.u = dalloc((M + 1) * n);
  L.unew = dalloc((M + 1) * n);
  L.f = dalloc(M * n);
  L.C = dalloc((M + 1) * n);
  L.Cnew = dalloc((M + 1) * n);
  L.X = dalloc(M * n);
  L.gf = dalloc(M * n);
  L.v = dalloc((M + 1) * n);
  L.r = dalloc(M * n);
  L.q = dalloc(M * n);
  L.b = dalloc(n);
  L.y = dalloc(n);
  L.t1 = dalloc(n);
  L.t2 = dalloc(n);
  L.t3 = dalloc(n);
  L.diag = dalloc(n);
  L.cr = dalloc(n);
  L.cz = dalloc(n);
  L.cp = dalloc(n);
  L.cs = dalloc(n);
  L.cw = dalloc(n);
  L.trace = dalloc((size_t)L.nv * L.E * 2 * pr.dim * g.nf);
  L.idg = dalloc(L.np);
  L.idgc64.tab = dalloc((size_t)Level::IdgCache::kSlots * L.np);
  if (L.nv == 1) {  // the persistent PCG serves scalar equations only
    const size_t words = (size_t)2 * 2 * L.nv * L.E * 2 * pr.dim * g.nf;
    void* pz = nullptr;
    void* pt = nullptr;
    if (hipMalloc(&pz, words * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&pt, words * sizeof(unsigned long long)) != hipSuccess) {
      if (pz) (void)hipFree(pz);
      fail(SISDC_ENOMEM, "hipMalloc failed");
    }
    L.fz = (unsigned long long*)pz;
    L.ft = (unsigned long long*)pt;
    L.fwords = words;
    HIPCHECK(hipMemset(L.fz, 0, words * sizeof(unsigned long long)));
    HIPCHECK(hipMemset(L.ft, 0, words * sizeof(unsigned long long)));
  }
  L.r32 = falloc(n);  // FP32 staging of residuals (mixed solves, learned guess)
  if (h->meth.precision == SISDC_MIXED) {
    std::vector<float> t32(tab.begin(), tab.end());
    L.tab32 = falloc(t32.size());
    HIPCHECK(hipMemcpy(L.tab32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
    L.ub32 = falloc(L.vs);
    L.e32 = falloc(n);
    L.cr32 = falloc(n);
    L.cz32 = falloc(n);
    L.cp32 = falloc(n);
    L.cs32 = falloc(n);
    L.cw32 = falloc(n);
    L.diag32 = falloc(n);
    L.trace32 = falloc((size_t)L.nv * L.E * 2 * pr.dim * g.nf);
    L.idg32 = falloc(L.np);
    L.idgc32.tab = falloc((size_t)Level::IdgCache::kSlots * L.np);
  }
  HIPCHECK(hipMemset(L.u, 0, (M + 1) * n * sizeof(double)));
  HIPCHECK(hipMemset(L.gf, 0, M * n * sizeof(double)));
}

void free_level(Level& L) {
  double* ptrs[] = {L.tab, L.mw, L.u, L.unew, L.f, L.C, L.Cnew, L.X, L.gf, L.v, L.r, L.q, L.b, L.y,
                    L.t1, L.t2, L.t3, L.diag, L.cr, L.cz, L.cp, L.cs, L.cw, L.trace, L.idg, L.fds};
  for (double* p : ptrs)
    if (p) (void)hipFree(p);
  if (L.fz) (void)hipFree(L.fz);
  if (L.ft) (void)hipFree(L.ft);
  if (L.idgc64.tab) (void)hipFree(L.idgc64.tab);
  if (L.idgc32.tab) (void)hipFree(L.idgc32.tab);
  float* fptrs[] = {L.idg32, L.tab32, L.ub32, L.r32, L.e32, L.cr32, L.cz32, L.cp32, L.cs32, L.cw32, L.diag32, L.trace32,
                    L.net.theta, L.net.m, L.net.v, L.net.g, L.net.Xd, L.net.Td, L.net.Z1, L.net.A1, L.net.Z2,
                    L.net.A2, L.net.Y, L.net.dY, L.net.dA, L.net.dZ, L.net.Xi, L.net.A1i, L.net.A2i, L.net.Yi,
                    L.net.Xs, L.net.Ts};
  double* dptrs[] = {L.net.nrm, L.net.xnew, L.net.x0h, L.net.r0h, L.net.lossp};
  for (double* p : dptrs)
    if (p) (void)hipFree(p);
  for (float* p : fptrs)
    if (p) (void)hipFree(p);
}

// L^2 projection onto the coarse polynomials of an element, one axis:
// P = (I^T W_f I)^-1 I^T W_f (n1c x n1f), the coarse mass by the fine GLL
// quadrature (exact for Pc < Pf); Gaussian elimination with partial pivoting.
std::vector<double> l2_projection(const std::vector<double>& I, const std::vector<double>& wf, int n1f, int n1c) {
  std::vector<double> A(n1c * n1c, 0.0), B(n1c * n1f, 0.0);
  for (int a = 0; a < n1c; ++a) {
    for (int b = 0; b < n1c; ++b)
      for (int i = 0; i < n1f; ++i) A[a * n1c + b] += I[i * n1c + a] * wf[i] * I[i * n1c + b];
    for (int i = 0; i < n1f; ++i) B[a * n1f + i] = I[i * n1c + a] * wf[i];
  }
  for (int k = 0; k < n1c; ++k) {
    int piv = k;
    for (int r = k + 1; r < n1c; ++r)
      if (std::fabs(A[r * n1c + k]) > std::fabs(A[piv * n1c + k])) piv = r;
    if (A[piv * n1c + k] == 0.0) fail(SISDC_EINVAL, "singular coarse mass matrix");
    if (piv != k) {
      for (int c = 0; c < n1c; ++c) std::swap(A[k * n1c + c], A[piv * n1c + c]);
      for (int c = 0; c < n1f; ++c) std::swap(B[k * n1f + c], B[piv * n1f + c]);
    }
    for (int r = k + 1; r < n1c; ++r) {
      const double f = A[r * n1c + k] / A[k * n1c + k];
      for (int c = k; c < n1c; ++c) A[r * n1c + c] -= f * A[k * n1c + c];
      for (int c = 0; c < n1f; ++c) B[r * n1f + c] -= f * B[k * n1f + c];
    }
  }
  for (int k = n1c - 1; k >= 0; --k)
    for (int c = 0; c < n1f; ++c) {
      double v = B[k * n1f + c];
      for (int j = k + 1; j < n1c; ++j) v -= A[k * n1c + j] * B[j * n1f + c];
      B[k * n1f + c] = v / A[k * n1c + k];
    }
  return B;
}

// 2:1 h-coarsening, one axis, on the pair of fine elements that a coarse
// element fuses (2 n1f nodes, left child first; reference coordinates
// xi_c = (xi_f - 1)/2 on the left child, (xi_f + 1)/2 on the right):
//   I (2 n1f x n1c): each child evaluates the coarse polynomial at its nodes;
//   P (n1c x 2 n1f), embedded interpolation: a coarse node takes the value of
//     the child that holds it, after the jump J between the children (right
//     child's shared-face value minus the left's) is blended away linearly:
//     + J/2 (xi_c + 1) on the left child, - J/2 (1 - xi_c) on the right, so
//     the shared centre gets the mean of both;
//   P, L^2: (I^T W I)^-1 I^T W, W = diag(w_f / 2, w_f / 2).
void h_transfer_tables(const Level& F, const Level& Cc, int projection, std::vector<double>& I,
                       std::vector<double>& P) {
  const int nf = F.n1, nc = Cc.n1;
  std::vector<double> tl(nf), tr(nf);
  for (int i = 0; i < nf; ++i) {
    tl[i] = 0.5 * (F.xg[i] - 1.0);
    tr[i] = 0.5 * (F.xg[i] + 1.0);
  }
  const std::vector<double> Il = lagrange(Cc.xg, tl), Ir = lagrange(Cc.xg, tr);  // (nf x nc) each
  I.assign(2 * nf * nc, 0.0);
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j < nc; ++j) {
      I[i * nc + j] = Il[i * nc + j];
      I[(nf + i) * nc + j] = Ir[i * nc + j];
    }
  if (projection == SISDC_PROJ_L2) {
    std::vector<double> w2(2 * nf);
    for (int i = 0; i < nf; ++i) w2[i] = w2[nf + i] = 0.5 * F.wg[i];
    P = l2_projection(I, w2, 2 * nf, nc);
    return;
  }
  P.assign(nc * 2 * nf, 0.0);
  for (int j = 0; j < nc; ++j) {
    const double x = Cc.xg[j];
    double* row = &P[j * 2 * nf];
    if (x == 0.0) {  // the shared centre
      row[nf - 1] += 0.5;
      row[nf] += 0.5;
      continue;
    }
    const std::vector<double> t{x < 0.0 ? 2.0 * x + 1.0 : 2.0 * x - 1.0};
    const std::vector<double> l = lagrange(F.xg, t);  // (1 x nf)
    const int off = x < 0.0 ? 0 : nf;
    for (int i = 0; i < nf; ++i) row[off + i] = l[i];
    const double phi = x < 0.0 ? 0.5 * (x + 1.0) : -0.5 * (1.0 - x);  // weight of J
    row[nf] += phi;
    row[nf - 1] -= phi;
  }
}

void build_transfer(Transfer& T, const Level& F, const Level& Cc, int projection, int formulation) {
  T.h = Cc.E != F.E;
  const int nfi = T.h ? 2 * F.n1 : F.n1;  // fine-side length of the 1-D operators
  std::vector<double> I, P;
  if (T.h) {
    h_transfer_tables(F, Cc, projection, I, P);
  } else {
    I = lagrange(Cc.xg, F.xg);  // (n1f x n1c)
    P = projection == SISDC_PROJ_L2 ? l2_projection(I, F.wg, F.n1, Cc.n1) : lagrange(F.xg, Cc.xg);  // (n1c x n1f)
  }
  std::vector<double> R(Cc.n1 * nfi);
  for (int i = 0; i < nfi; ++i)
    for (int j = 0; j < Cc.n1; ++j) R[j * nfi + i] = I[i * Cc.n1 + j];
  T.Ix = dalloc(I.size());
  T.Px = dalloc(P.size());
  T.Rx = dalloc(R.size());
  HIPCHECK(hipMemcpy(T.Ix, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(T.Px, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(T.Rx, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice));
  T.It = lagrange(Cc.tau, F.tau);  // (Mf x Mc)
  T.Pt = lagrange(F.tau, Cc.tau);  // (Mc x Mf)
  // Residual restriction in time.  The non-incremental (zero-to-node) form
  // (Sec. 4, eq. ml-sdc:non-incremental:matrix) restricts the node sums
  // r0n = C_f r and its coarse FAS term is g0n = C_c g, C the lower-
  // triangular matrix of ones; in node-to-node variables that is the
  // restriction C_c^-1 I_t^T C_f: row mc of I_t^T C_f minus row mc - 1.
  const int Mf = F.M, Mc = Cc.M;
  std::vector<double> RC(Mc * Mf, 0.0);  // I_t^T C_f: sum over fine nodes k >= i of It[k][j]
  for (int j = 0; j < Mc; ++j)
    for (int i = 0; i < Mf; ++i) {
      double acc = 0.0;
      for (int k = i; k < Mf; ++k) acc += T.It[k * Mc + j];
      RC[j * Mf + i] = acc;
    }
  T.Rt.assign(Mc * Mf, 0.0);
  for (int j = 0; j < Mc; ++j)
    for (int i = 0; i < Mf; ++i)
      T.Rt[j * Mf + i] = formulation == SISDC_NONINCREMENTAL
                             ? RC[j * Mf + i] - (j > 0 ? RC[(j - 1) * Mf + i] : 0.0)
                             : T.It[i * Mc + j];
}

void validate(const sisdc_problem* p, const sisdc_method* m) {
  if (!p || !m) fail(SISDC_EINVAL, "null problem or method");
  if (p->dim != 2 && p->dim != 3) fail(SISDC_EINVAL, "dim must be 2 or 3");
  for (int d = 0; d < p->dim; ++d) {
    if (p->n_elem[d] < 1) fail(SISDC_EINVAL, "n_elem must be >= 1");
    if (!(p->hi[d] > p->lo[d])) fail(SISDC_EINVAL, "hi must exceed lo");
  }
  if (p->eq < SISDC_EQ_CONVDIFF || p->eq > SISDC_EQ_NS) fail(SISDC_EINVAL, "unknown equation");
  const bool sys = p->eq == SISDC_EQ_EULER || p->eq == SISDC_EQ_NS;
  if (sys && !(p->gamma > 1.0)) fail(SISDC_EINVAL, "gamma must exceed 1");
  if (!sys && !(p->nu >= 0.0)) fail(SISDC_EINVAL, "nu must be >= 0");
  if (p->eq == SISDC_EQ_NS && (!(p->mu >= 0.0) || !(p->Pr > 0.0))) fail(SISDC_EINVAL, "NS needs mu >= 0, Pr > 0");
  if (m->n_levels < 1 || m->n_levels > 3) fail(SISDC_EINVAL, "n_levels must be 1..3");
  for (int l = 0; l < m->n_levels; ++l) {
    if (m->P[l] < 1 || m->P[l] > kMaxP) fail(SISDC_EINVAL, "P must be 1..8");
    if (m->M[l] < 1 || m->M[l] > 8) fail(SISDC_EINVAL, "M must be 1..8");
    if (l > 0 && m->P[l] > m->P[l - 1]) fail(SISDC_EINVAL, "coarser levels need P <= finer P");
  }
  if (m->integrator != SISDC_SI2 && m->integrator != SISDC_SI1 && m->integrator != SISDC_IMEX_EULER)
    fail(SISDC_EINVAL, "integrator");
  if (m->projection != SISDC_PROJ_INTERP && m->projection != SISDC_PROJ_L2) fail(SISDC_EINVAL, "projection");
  if (m->formulation != SISDC_INCREMENTAL && m->formulation != SISDC_NONINCREMENTAL) fail(SISDC_EINVAL, "formulation");
  if (m->nodes != SISDC_NODES_RADAU_RIGHT && m->nodes != SISDC_NODES_LOBATTO) fail(SISDC_EINVAL, "nodes");
  if (m->h_coarsen[0] != 0) fail(SISDC_EINVAL, "h_coarsen[0] must be 0 (the finest level is not coarsened)");
  {
    int ne[3] = {p->n_elem[0], p->n_elem[1], p->dim == 3 ? p->n_elem[2] : 1};
    for (int l = 1; l < m->n_levels; ++l) {
      if (m->h_coarsen[l] != 0 && m->h_coarsen[l] != 1) fail(SISDC_EINVAL, "h_coarsen must be 0 or 1");
      if (!m->h_coarsen[l]) continue;
      for (int d = 0; d < p->dim; ++d) {
        if (ne[d] % 2 != 0) fail(SISDC_EINVAL, "h-coarsening needs an even number of elements along every axis");
        ne[d] /= 2;
      }
      if (p->dim == 3 && m->P[l - 1] > 6) fail(SISDC_EINVAL, "3-D h-coarsening supports fine degrees up to 6");
    }
  }
  if (m->nodes == SISDC_NODES_LOBATTO)
    for (int l = 0; l < m->n_levels; ++l)
      if (m->M[l] < 2) fail(SISDC_EINVAL, "Lobatto nodes need M >= 2 on every level");
  if (m->start < SISDC_START_CASCADE || m->start > SISDC_START_CONSTANT) fail(SISDC_EINVAL, "start");
  if (m->n_iter < 0 || m->n_coarse_sweeps < 0) fail(SISDC_EINVAL, "negative sweep count");
  if (m->conserve != 0 && m->conserve != 1) fail(SISDC_EINVAL, "conserve must be 0 or 1");
  if (m->precond != SISDC_PRECOND_JACOBI && m->precond != SISDC_PRECOND_FDS) fail(SISDC_EINVAL, "precond");
  if (!(m->cg_rtol > 0.0) || m->cg_maxit < 1) fail(SISDC_EINVAL, "cg_rtol > 0 and cg_maxit >= 1 required");
  if (m->precision != SISDC_FP64 && m->precision != SISDC_MIXED) fail(SISDC_EINVAL, "precision");
  if (p->stack < 0) fail(SISDC_EINVAL, "stack must be >= 0");
  if (p->stack > 1) {
    if (sys) fail(SISDC_EINVAL, "stacked ensembles take scalar equations (CONVDIFF, BURGERS)");
    if (m->conserve) fail(SISDC_EINVAL, "stacked ensembles need conserve = 0 (the shift is one constant per component)");
    for (int l = 1; l < m->n_levels; ++l)
      if (m->h_coarsen[l]) fail(SISDC_EINVAL, "stacked ensembles take no h_coarsen");
    if ((long)p->stack * p->n_elem[p->dim - 1] > (1L << 20)) fail(SISDC_EINVAL, "stack too large");
  }
  if (!(m->av_c >= 0.0)) fail(SISDC_EINVAL, "av_c must be >= 0");
  if (m->av_c > 0.0) {
    if (!(m->av_kappa > 0.0)) fail(SISDC_EINVAL, "artificial viscosity needs av_kappa > 0");
    if (m->precision != SISDC_FP64) fail(SISDC_EINVAL, "artificial viscosity runs with FP64 solves");
    for (int l = 1; l < m->n_levels; ++l)
      if (m->h_coarsen[l]) fail(SISDC_EINVAL, "artificial viscosity needs the same elements on every level");
  }
  if (m->cg_variant != SISDC_CG_AUTO && m->cg_variant != SISDC_CG_MULTI_KERNEL &&
      m->cg_variant != SISDC_CG_PERSISTENT_COOPERATIVE)
    fail(SISDC_EINVAL, "cg_variant");
}

// Caller pointer -> device pointer (host data staged through h->io).
const double* dev_in(sisdc_handle* h, const double* p, long n, int mem, double* stage) {
  if (mem == SISDC_MEM_DEVICE) return p;
  if (mem != SISDC_MEM_HOST) fail(SISDC_EINVAL, "mem must be SISDC_MEM_HOST or SISDC_MEM_DEVICE");
  HIPCHECK(hipMemcpyAsync(stage, p, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
  return stage;
}

void dev_out(sisdc_handle* h, double* user, const double* src, long n, int mem) {
  if (mem == SISDC_MEM_DEVICE) {
    if (user != src) copy_d2d(h, user, src, n);
  } else {
    HIPCHECK(hipMemcpyAsync(user, src, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHECK(hipStreamSynchronize(h->stream));
}

Level& level_at(sisdc_handle* h, int level) {
  if (!h) fail(SISDC_EINVAL, "null handle");
  if (level < 0 || level >= (int)h->lv.size()) fail(SISDC_EINVAL, "level out of range");
  return h->lv[level];
}

template <class F>
int guard(F&& f) {
  try {
    f();
    g_last_error.clear();
    return SISDC_OK;
  } catch (const Err& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return SISDC_ENOMEM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return SISDC_EDEVICE;
  }
}

}  // namespace

namespace {

// ------------------------------------------------------------------ network helpers
// SplitMix64 (Vigna): k-th output of the generator seeded with `seed`.
uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void net_free(Level& L) {
  auto& N = L.net;
  float* f[] = {N.theta, N.m, N.v, N.g, N.Xd, N.Td, N.Z1, N.A1, N.Z2, N.A2, N.Y, N.dY, N.dA, N.dZ, N.Xi, N.A1i,
                N.A2i, N.Yi, N.Xs, N.Ts};
  for (float* p : f)
    if (p) (void)hipFree(p);
  double* d[] = {N.nrm, N.xnew, N.x0h, N.r0h, N.lossp};
  for (double* p : d)
    if (p) (void)hipFree(p);
  N = Level::Net{};
}

// one Adam step on rows X, T (device, FP32); loss partials into lossp
void net_train_batch(sisdc_handle* h, Level& L, const float* X, const float* T, int rows, double lr, double* lossp) {
  auto& N = L.net;
  hipStream_t s = h->stream;
  HIPCHECK(mlp_forward(N.sh, N.theta, X, rows, N.Z1, N.A1, N.Z2, N.A2, N.Y, 0, s));
  HIPCHECK(mlp_backward(N.sh, N.theta, X, T, rows, N.Z1, N.A1, N.Z2, N.A2, N.Y, N.dY, N.dA, N.dZ, N.g, lossp, s));
  N.step += 1;
  HIPCHECK(launch_adam(N.theta, N.m, N.v, N.g, N.sh.params(), (float)lr, N.step, s));
}

Level::Net& net_of(sisdc_handle* h, int level) {
  Level& L = level_at(h, level);
  if (!L.net.on) fail(SISDC_ESTATE, "sisdc_net_init must come first for this level");
  return L.net;
}

}  // namespace

// ==================================================================== C ABI
extern "C" {

const char* sisdc_last_error(void) { return g_last_error.c_str(); }

int sisdc_create(const sisdc_problem* prob, const sisdc_method* meth, void* hip_stream, sisdc_handle** out) {
  if (!out) {
    g_last_error = "null output pointer";
    return SISDC_EINVAL;
  }
  *out = nullptr;
  sisdc_handle* h = nullptr;
  int rc = guard([&] {
    validate(prob, meth);
    h = new sisdc_handle();
    h->prob = *prob;
    h->meth = *meth;
    h->stream = (hipStream_t)hip_stream;
    h->ctau = meth->c_tau > 0.0 ? meth->c_tau : 2.0;
    h->eq.eq = prob->eq;
    const bool sys = prob->eq == SISDC_EQ_EULER || prob->eq == SISDC_EQ_NS;
    h->eq.nv = sys ? prob->dim + 2 : 1;
    for (int d = 0; d < 3; ++d) h->eq.a[d] = d < prob->dim ? prob->a[d] : 0.0;
    h->eq.nu = sys ? 0.0 : prob->nu;
    h->eq.gamma = prob->gamma;
    h->eq.R = prob->R > 0.0 ? prob->R : 1.0;
    h->eq.mu = prob->eq == SISDC_EQ_NS ? prob->mu : 0.0;
    h->eq.lam_T = prob->eq == SISDC_EQ_NS ? prob->mu * (prob->gamma * h->eq.R / (prob->gamma - 1.0)) / prob->Pr : 0.0;
    h->lv.resize(meth->n_levels);
    // elements per axis of each level: halved where the level is 2:1 h-coarsened
    int ne[3][3];
    for (int d = 0; d < 3; ++d) ne[0][d] = d < prob->dim ? prob->n_elem[d] : 1;
    if (prob->stack > 1) ne[0][prob->dim - 1] *= prob->stack;  // the instances, one after another
    for (int l = 1; l < meth->n_levels; ++l)
      for (int d = 0; d < 3; ++d) ne[l][d] = (meth->h_coarsen[l] && d < prob->dim) ? ne[l - 1][d] / 2 : ne[l - 1][d];
    for (int l = 0; l < meth->n_levels; ++l) build_level(h, h->lv[l], meth->P[l], meth->M[l], ne[l]);
    h->tr.resize(meth->n_levels > 1 ? meth->n_levels - 1 : 0);
    for (int l = 0; l + 1 < meth->n_levels; ++l) build_transfer(h->tr[l], h->lv[l], h->lv[l + 1], meth->projection, meth->formulation);
    h->partials = dalloc((size_t)7 * kElemCap);
    h->cons = dalloc((size_t)15 * kElemCap + 64);
    h->ir_tot = dalloc(2);
    h->gtot = dalloc(4);
    void* pn = nullptr;
    if (hipMalloc(&pn, 64) != hipSuccess) fail(SISDC_ENOMEM, "hipMalloc failed");
    h->nrej = (int*)pn;
    HIPCHECK(hipMemset(h->nrej, 0, 64));
    void* pf = nullptr;
    if (hipMalloc(&pf, 7 * kElemCap * sizeof(float) + 64) != hipSuccess) fail(SISDC_ENOMEM, "hipMalloc failed");
    h->partials32 = (float*)pf;
    h->alpha32 = h->partials32 + 7 * kElemCap;
    h->alpha = dalloc(2);
    // the result record and the convergence word in one block, at the
    // offsets of their pinned host mirrors, so one copy brings both back
    void* pr = nullptr;
    if (hipMalloc(&pr, 256) != hipSuccess) fail(SISDC_ENOMEM, "hipMalloc failed");
    HIPCHECK(hipMemset(pr, 0, 256));
    h->res = (CGRes*)pr;
    h->done_gen = (int*)((char*)pr + kDoneOffset);
    void* hp = nullptr;
    if (hipHostMalloc(&hp, 256) != hipSuccess) fail(SISDC_ENOMEM, "hipHostMalloc failed");
    h->hres = (CGRes*)hp;
    h->hdone = (int*)((char*)hp + kDoneOffset);
    h->hlam = (double*)((char*)hp + 192);
    h->hir_tot = (double*)((char*)hp + 208 + 16);
    h->hnrej = (int*)((char*)hp + 248);
    h->lam_dev = dalloc(2);
    h->pcap = 1024;
    void* pp = nullptr;
    if (hipMalloc(&pp, (size_t)2 * 16 * h->pcap * sizeof(unsigned long long)) != hipSuccess)
      fail(SISDC_ENOMEM, "hipMalloc failed");
    h->ppart = (unsigned long long*)pp;
    HIPCHECK(hipMemset(h->ppart, 0, (size_t)2 * 16 * h->pcap * sizeof(unsigned long long)));
    void* pb = nullptr;
    if (hipMalloc(&pb, 512) != hipSuccess) fail(SISDC_ENOMEM, "hipMalloc failed");
    h->bar = (unsigned*)pb;
    HIPCHECK(hipMemset(h->bar, 0, 512));
    void* prr = nullptr;
    if (hipMalloc(&prr, kRing * sizeof(CGRes)) != hipSuccess) fail(SISDC_ENOMEM, "hipMalloc failed");
    h->ring = (CGRes*)prr;
    void* hrr = nullptr;
    if (hipHostMalloc(&hrr, kRing * sizeof(CGRes)) != hipSuccess) fail(SISDC_ENOMEM, "hipHostMalloc failed");
    h->hring = (CGRes*)hrr;
    h->av = meth->av_c > 0.0;
    if (h->av) {
      Level& F = h->lv[0];
      h->eps = dalloc(F.E);
      HIPCHECK(hipMemset(h->eps, 0, F.E * sizeof(double)));
      const std::vector<double> A = legendre_analysis(F.P, F.xg, F.wg);
      h->av_tab = dalloc(A.size());
      HIPCHECK(hipMemcpy(h->av_tab, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    for (auto& L : h->lv)
      L.persistent = persistent_fits(h, L, meth->cg_variant);
    h->state = dalloc(h->lv[0].vlen);
    size_t io = 0;
    for (auto& L : h->lv) io = std::max(io, (size_t)(L.M + 1) * L.vlen);
    h->io_len = io;
    h->io = dalloc(io);
    HIPCHECK(hipGetDevice(&h->dev));
    porder_register(h->dev, h->stream);
    h->registered = true;
  });
  if (rc != SISDC_OK) {
    if (h) sisdc_destroy(h);
    return rc;
  }
  *out = h;
  return SISDC_OK;
}

int sisdc_destroy(sisdc_handle* h) {
  if (!h) return SISDC_OK;
  (void)hipDeviceSynchronize();
  if (h->registered) porder_unregister(h->dev, h->stream);
  graph_drop(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (auto& L : h->lv) {
    net_free(L);
    free_level(L);
  }
  for (auto& T : h->tr) {
    if (T.Ix) (void)hipFree(T.Ix);
    if (T.Px) (void)hipFree(T.Px);
    if (T.Rx) (void)hipFree(T.Rx);
  }
  if (h->partials) (void)hipFree(h->partials);
  if (h->cons) (void)hipFree(h->cons);
  if (h->alpha) (void)hipFree(h->alpha);
  if (h->partials32) (void)hipFree(h->partials32);
  if (h->ir_tot) (void)hipFree(h->ir_tot);
  if (h->gtot) (void)hipFree(h->gtot);
  if (h->nrej) (void)hipFree(h->nrej);
  if (h->res) (void)hipFree(h->res);  // the block that holds done_gen too
  if (h->hres) (void)hipHostFree(h->hres);
  if (h->lam_dev) (void)hipFree(h->lam_dev);
  if (h->ppart) (void)hipFree(h->ppart);
  if (h->bar) (void)hipFree(h->bar);
  if (h->ring) (void)hipFree(h->ring);
  if (h->hring) (void)hipHostFree(h->hring);
  for (hipEvent_t ev : h->pev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : h->mev) (void)hipEventDestroy(ev);
  if (h->state) (void)hipFree(h->state);
  if (h->eps) (void)hipFree(h->eps);
  if (h->av_tab) (void)hipFree(h->av_tab);
  if (h->io) (void)hipFree(h->io);
  delete h;
  return SISDC_OK;
}

int sisdc_level_info(const sisdc_handle* hc, int level, int* n_elem_total, int* nodes_per_elem, int* n_var,
                     int* M) {
  return guard([&] {
    sisdc_handle* h = const_cast<sisdc_handle*>(hc);
    Level& L = level_at(h, level);
    if (n_elem_total) *n_elem_total = L.E;
    if (nodes_per_elem) *nodes_per_elem = L.np;
    if (n_var) *n_var = L.nv;
    if (M) *M = L.M;
  });
}

int sisdc_node_coords(sisdc_handle* h, int level, double* x, int mem) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!x) fail(SISDC_EINVAL, "null output");
    const int dim = h->prob.dim;
    std::vector<double> c((size_t)dim * L.E * L.np);
    for (int e = 0; e < L.E; ++e) {
      int ec[3] = {e % L.g.ne[0], (e / L.g.ne[0]) % L.g.ne[1], dim == 3 ? e / (L.g.ne[0] * L.g.ne[1]) : 0};
      for (int n = 0; n < L.np; ++n) {
        int ic[3] = {n % L.n1, (n / L.n1) % L.n1, n / (L.n1 * L.n1)};
        for (int d = 0; d < dim; ++d)
          c[((size_t)d * L.E + e) * L.np + n] =
              h->prob.lo[d] + L.g.h[d] * ((d == dim - 1 ? ec[d] % L.g.wl : ec[d]) + 0.5 * (L.xg[ic[d]] + 1.0));
      }
    }
    if (mem == SISDC_MEM_HOST) {
      std::memcpy(x, c.data(), c.size() * sizeof(double));
    } else {
      HIPCHECK(hipMemcpy(x, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  });
}

int sisdc_set_state(sisdc_handle* h, const double* u0, int mem) {
  return guard([&] {
    Level& L = level_at(h, 0);
    if (!u0) fail(SISDC_EINVAL, "null state");
    const double* d = dev_in(h, u0, L.vlen, mem, h->io);
    copy_d2d(h, h->state, d, L.vlen);
    copy_d2d(h, L.um(0), d, L.vlen);
    HIPCHECK(hipStreamSynchronize(h->stream));
    h->have_state = true;
  });
}

int sisdc_get_state(sisdc_handle* h, double* u, int mem) {
  return guard([&] {
    Level& L = level_at(h, 0);
    if (!u) fail(SISDC_EINVAL, "null output");
    dev_out(h, u, h->state, L.vlen, mem);
  });
}

int sisdc_get_level(sisdc_handle* h, int level, double* u, int mem) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!u) fail(SISDC_EINVAL, "null output");
    dev_out(h, u, L.u, (long)(L.M + 1) * L.vlen, mem);
  });
}

int sisdc_set_level(sisdc_handle* h, int level, const double* u, int mem) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!u) fail(SISDC_EINVAL, "null input");
    const long n = (long)(L.M + 1) * L.vlen;
    const double* d = dev_in(h, u, n, mem, h->io);
    copy_d2d(h, L.u, d, n);
    HIPCHECK(hipStreamSynchronize(h->stream));
    L.stale = true;
  });
}

int sisdc_get_fas(sisdc_handle* h, int level, double* g, int mem) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!g) fail(SISDC_EINVAL, "null output");
    if (!L.has_g) {
      HIPCHECK(hipMemsetAsync(L.gf, 0, (size_t)L.M * L.vlen * sizeof(double), h->stream));
    }
    dev_out(h, g, L.gf, (long)L.M * L.vlen, mem);
  });
}

int sisdc_set_fas(sisdc_handle* h, int level, const double* g, int mem) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!g) {
      L.has_g = false;
      return;
    }
    const long n = (long)L.M * L.vlen;
    const double* d = dev_in(h, g, n, mem, h->io);
    copy_d2d(h, L.gf, d, n);
    HIPCHECK(hipStreamSynchronize(h->stream));
    L.has_g = true;
  });
}

int sisdc_update_step_params(sisdc_handle* h, double* lam_out) {
  return guard([&] {
    level_at(h, 0);
    update_lam(h);
    if (lam_out) *lam_out = h->lam;
  });
}

int sisdc_step(sisdc_handle* h, double t, double dt, sisdc_stats* st) {
  (void)t;
  return guard([&] {
    level_at(h, 0);
    if (!h->have_state) fail(SISDC_ESTATE, "sisdc_set_state must precede sisdc_step");
    if (!(dt > 0.0)) fail(SISDC_EINVAL, "dt must be positive");
    h->st = sisdc_stats{};
    h->g_last = h->graph_on && graph_step(h, dt);
    if (!h->g_last) do_step(h, dt);
    if (st) *st = h->st;
    if (h->st.not_converged) fail(SISDC_ENOTCONV, "a Helmholtz solve reached cg_maxit");
  });
}

int sisdc_predict(sisdc_handle* h, int level, double dt, sisdc_stats* st) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!(dt > 0.0)) fail(SISDC_EINVAL, "dt must be positive");
    h->st = sisdc_stats{};
    predictor(h, L, dt);
    if (level == 0) h->st.fine_sweeps += 1;
    drain(h);
    HIPCHECK(hipStreamSynchronize(h->stream));
    if (st) *st = h->st;
  });
}

int sisdc_sweep(sisdc_handle* h, int level, double dt, const double* g, int mem, sisdc_stats* st) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!(dt > 0.0)) fail(SISDC_EINVAL, "dt must be positive");
    h->st = sisdc_stats{};
    if (g) {
      const long n = (long)L.M * L.vlen;
      const double* d = dev_in(h, g, n, mem, h->io);
      if (d != L.gf) copy_d2d(h, L.gf, d, n);
      L.has_g = true;
    }
    sweep(h, L, dt, L.has_g ? L.gf : nullptr);
    if (level == 0) h->st.fine_sweeps += 1;
    drain(h);
    HIPCHECK(hipStreamSynchronize(h->stream));
    if (st) *st = h->st;
  });
}

int mlsdc_vcycle(sisdc_handle* h, int top_level, double dt, sisdc_stats* st) {
  return guard([&] {
    level_at(h, top_level);
    if (top_level >= (int)h->lv.size() - 1) fail(SISDC_EINVAL, "top_level must have a coarser level");
    if (!(dt > 0.0)) fail(SISDC_EINVAL, "dt must be positive");
    h->st = sisdc_stats{};
    vcycle(h, top_level, dt);
    drain(h);
    HIPCHECK(hipStreamSynchronize(h->stream));
    if (st) *st = h->st;
  });
}

int helmholtz_solve(sisdc_handle* h, int level, double dt_m, const double* coef_state, const double* b, double* x,
                    int mem, double rtol, int maxit, sisdc_solve_stats* st) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!b || !x) fail(SISDC_EINVAL, "null b or x");
    if (!(dt_m >= 0.0)) fail(SISDC_EINVAL, "dt_m must be >= 0");
    if (h->eq.eq == EQ_BURGERS && !coef_state) fail(SISDC_EINVAL, "Burgers needs coef_state");
    const long n = L.vlen;
    const double* db = dev_in(h, b, n, mem, L.t1);
    const double* dub = coef_state ? dev_in(h, coef_state, n, mem, L.t2) : nullptr;
    double* dx = x;
    if (mem == SISDC_MEM_HOST) {
      HIPCHECK(hipMemcpyAsync(L.y, x, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
      dx = L.y;
    }
    copy_d2d(h, L.b, db, n);
    CoefP cf = coef_for(h, L, dt_m, dub);
    h->st = sisdc_stats{};
    sisdc_solve_stats r = cg_solve(h, L, cf, dt_m, L.b, dx, rtol > 0 ? rtol : h->meth.cg_rtol,
                                   maxit > 0 ? maxit : h->meth.cg_maxit);
    drain(h);
    if (r.iters < 0) {
      r.iters = (int)h->st.cg_iters;
      r.converged = h->st.not_converged == 0;
      r.rel_residual = h->st.max_rel_residual;
    }
    if (mem == SISDC_MEM_HOST) dev_out(h, x, dx, n, mem);
    if (st) *st = r;
    if (!r.converged) fail(SISDC_ENOTCONV, "CG reached maxit before the tolerance");
  });
}

int helmholtz_solve_noalloc(sisdc_handle* h, int level, double dt_m, const double* coef_state, const double* b,
                            double* x, double rtol, int maxit, sisdc_solve_stats* st) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!b || !x) fail(SISDC_EINVAL, "null b or x");
    if (!(dt_m >= 0.0)) fail(SISDC_EINVAL, "dt_m must be >= 0");
    if (h->eq.eq == EQ_BURGERS && !coef_state) fail(SISDC_EINVAL, "Burgers needs coef_state");
    int cur = -1;
    HIPCHECK(hipGetDevice(&cur));
    if (cur != h->dev) fail(SISDC_EINVAL, "the handle's device must be current");
    // carve the multi-kernel PCG's work space out of the device's static
    // scratch: r, z, p, s, w, diag (one level vector each), the face traces,
    // the inverse diagonal table, partial sums, step lengths, the result
    // record and the convergence word, each 256-byte aligned
    auto up = [](size_t n) { return (n + 255) & ~size_t(255); };
    const size_t vec = up((size_t)L.vlen * sizeof(double));
    const size_t trc = up((size_t)L.nv * L.E * 2 * L.g.dim * L.g.nf * sizeof(double));
    const size_t idg = up((size_t)L.np * sizeof(double));
    const size_t par = up((size_t)7 * kElemCap * sizeof(double));
    const size_t alp = up(2 * sizeof(double));
    const size_t rec = up(sizeof(CGRes)) + 256;  // the record, then the convergence word
    const size_t need = 6 * vec + trc + idg + par + alp + rec;
    if (need > kScratchBytes)
      fail(SISDC_EINVAL, "level too large for the static scratch: needs " + std::to_string(need) + " bytes, at most " +
                             std::to_string(kScratchBytes));
    void* base = nullptr;
    HIPCHECK(scratch_region(h->dev, &base));
    char* q = (char*)base;
    auto take = [&](size_t n) {
      char* r = q;
      q += n;
      return r;
    };
    CGBufs<double> B{};
    B.r = (double*)take(vec);
    B.z = (double*)take(vec);
    B.p = (double*)take(vec);
    B.s = (double*)take(vec);
    B.w = (double*)take(vec);
    B.diag = (double*)take(vec);
    B.trace = (double*)take(trc);
    B.idg = (double*)take(idg);
    B.partials = (double*)take(par);
    B.alpha = (double*)take(alp);
    char* recp = take(rec);
    B.res = (CGRes*)recp;
    B.done_gen = (int*)(recp + up(sizeof(CGRes)));
    B.tab = L.tab;
    // the previous call on this GPU may have left any id in the convergence
    // word and any record: clear both (a fill kernel, no memset node)
    HIPCHECK(launch_zero_scratch(recp, rec, h->stream));
    const CoefP cf = coef_for(h, L, dt_m, coef_state);
    h->st = sisdc_stats{};
    sisdc_solve_stats r = cg_multi<double>(h, L, B, cf, dt_m, b, x, rtol > 0 ? rtol : h->meth.cg_rtol,
                                           maxit > 0 ? maxit : h->meth.cg_maxit, false);
    account(h, r.iters, r.converged, r.rel_residual);
    HIPCHECK(hipStreamSynchronize(h->stream));
    if (st) *st = r;
    if (!r.converged) fail(SISDC_ENOTCONV, "CG reached maxit before the tolerance");
  });
}

int sisdc_apply(sisdc_handle* h, int op, int level, double dt_m, const double* in, const double* aux, double* out,
                int mem) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!in || !out) fail(SISDC_EINVAL, "null in or out");
    if (op == SISDC_OP_QUAD) {  // the node quadrature over M vectors (L.q is scratch between sweeps)
      const long n = (long)L.M * L.vlen;
      const double* din = dev_in(h, in, n, mem, h->io);
      double* dout = mem == SISDC_MEM_DEVICE ? out : L.q;
      LinCombMulti lc{};
      lc.nin = L.M;
      lc.nout = L.M;
      for (int i = 0; i < L.M; ++i) lc.x[i] = din + (long)i * L.vlen;
      for (int m = 0; m < L.M; ++m)
        for (int i = 0; i < L.M; ++i) lc.c[m][i] = dt_m * L.wnn[m * L.M + i];
      HIPCHECK(launch_lincomb_multi(dout, lc, L.vlen, h->stream));
      dev_out(h, out, dout, n, mem);
      return;
    }
    const bool down = op == SISDC_OP_PROJECT || op == SISDC_OP_RESTRICT;
    const bool up = op == SISDC_OP_INTERP;
    if ((down || up) && level + 1 >= (int)h->lv.size()) fail(SISDC_EINVAL, "transfer needs level+1");
    const Level& Lin = up ? h->lv[level + 1] : L;
    const Level& Lout = down ? h->lv[level + 1] : L;
    const double* din = dev_in(h, in, Lin.vlen, mem, Lin.t2);
    const double* daux = aux ? dev_in(h, aux, L.vlen, mem, L.t3) : nullptr;
    double* dout = mem == SISDC_MEM_DEVICE ? out : Lout.b;
    switch (op) {
      case SISDC_OP_MASS: lincomb(h, L, dout, {{1.0, din}}, {1}); break;
      case SISDC_OP_CONV: conv(h, L, din, dout); break;
      case SISDC_OP_FRHS:
        conv(h, L, din, L.t1);
        frhs_from_c(h, L, din, L.t1, dout);
        break;
      case SISDC_OP_SIPG: sipg(h, L, coef_for(h, L, dt_m, daux), din, dout, 0.0, 1.0); break;
      case SISDC_OP_HELM: sipg(h, L, coef_for(h, L, dt_m, daux), din, dout, 1.0, dt_m); break;
      case SISDC_OP_PROJECT: space_transfer(h, L, Lout, din, dout, h->tr[level].Px); break;
      case SISDC_OP_RESTRICT: space_transfer(h, L, Lout, din, dout, h->tr[level].Rx); break;
      case SISDC_OP_INTERP: space_transfer(h, Lin, L, din, dout, h->tr[level].Ix); break;
      case SISDC_OP_PRECOND: {
        const CoefP cf = coef_for(h, L, dt_m, daux);
        if (!sipg_iso_path(L.g, cf))
          fail(SISDC_EINVAL, "the block-Jacobi preconditioner needs an isotropic constant coefficient");
        HIPCHECK(launch_fds(din, dout, L.nv, L.g, L.fds, dt_m * cf.nu, nullptr, nullptr, nullptr, 0, h->stream));
        break;
      }
      default: fail(SISDC_EINVAL, "unknown op");
    }
    dev_out(h, out, dout, Lout.vlen, mem);
  });
}

int sisdc_collocation_residual(sisdc_handle* h, int level, double dt, double* out, int mem) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (!out) fail(SISDC_EINVAL, "null output");
    colloc_residual(h, L, dt, L.r, nullptr);
    dev_out(h, out, L.r, (long)L.M * L.vlen, mem);
  });
}

int sisdc_av_update(sisdc_handle* h) {
  return guard([&] {
    if (!h) fail(SISDC_EINVAL, "null handle");
    if (!h->av) fail(SISDC_EINVAL, "the method has no artificial viscosity (av_c = 0)");
    if (!h->have_state) fail(SISDC_ESTATE, "sisdc_set_state must precede sisdc_av_update");
    av_update(h, h->state);
    HIPCHECK(hipStreamSynchronize(h->stream));
  });
}

int sisdc_av_get(sisdc_handle* h, double* eps, int mem) {
  return guard([&] {
    if (!h) fail(SISDC_EINVAL, "null handle");
    if (!h->av) fail(SISDC_EINVAL, "the method has no artificial viscosity (av_c = 0)");
    if (!eps) fail(SISDC_EINVAL, "null output");
    dev_out(h, eps, h->eps, h->lv[0].E, mem);
  });
}

int sisdc_set_graph(sisdc_handle* h, int on) {
  return guard([&] {
    if (!h) fail(SISDC_EINVAL, "null handle");
    if (on != 0 && on != 1) fail(SISDC_EINVAL, "on must be 0 or 1");
    h->graph_on = on != 0;
    if (!on) graph_drop(h);
    h->g_refused_form = -1;
  });
}

int sisdc_graph_info(sisdc_handle* h, int* last_step_graphed, long long* captures, long long* replays) {
  return guard([&] {
    if (!h) fail(SISDC_EINVAL, "null handle");
    if (last_step_graphed) *last_step_graphed = h->g_last ? 1 : 0;
    if (captures) *captures = h->g_captures;
    if (replays) *replays = h->g_replays;
  });
}

int sisdc_pcg_timing(sisdc_handle* h, int on) {
  return guard([&] {
    if (!h) fail(SISDC_EINVAL, "null handle");
    drain(h);  // records launched before this call keep their own setting
    if (on && h->pev.empty()) {
      h->pev.resize(2 * kRing, nullptr);
      for (auto& ev : h->pev) HIPCHECK(hipEventCreate(&ev));
    }
    if (on) {
      h->pt_us.assign(h->lv.size(), 0.0);
      h->pt_n.assign(h->lv.size(), 0);
      h->pt_it.assign(h->lv.size(), 0);
      h->kt_us.assign(2 * h->lv.size(), 0.0);
      h->kt_n.assign(2 * h->lv.size(), 0);
      h->kt_stride = std::max(1, on);
      h->kt_solves = 0;
    }
    h->ptime = on != 0;
  });
}

int sisdc_cg_kernel_timing_get(sisdc_handle* h, int level, int kernel, long long* launches, double* total_us) {
  return guard([&] {
    level_at(h, level);
    if (kernel != SISDC_K_CG_UPDATE && kernel != SISDC_K_SIPG_APPLY) fail(SISDC_EINVAL, "kernel must be SISDC_K_CG_UPDATE or SISDC_K_SIPG_APPLY");
    const size_t k = 2 * (size_t)level + (kernel == SISDC_K_SIPG_APPLY ? 1 : 0);
    const bool have = k < h->kt_us.size();
    if (launches) *launches = have ? h->kt_n[k] : 0;
    if (total_us) *total_us = have ? h->kt_us[k] : 0.0;
  });
}

int sisdc_pcg_timing_get(sisdc_handle* h, int level, long long* launches, long long* iters, double* total_us) {
  return guard([&] {
    level_at(h, level);
    drain(h);
    const bool have = (size_t)level < h->pt_us.size();
    if (launches) *launches = have ? h->pt_n[level] : 0;
    if (iters) *iters = have ? h->pt_it[level] : 0;
    if (total_us) *total_us = have ? h->pt_us[level] : 0.0;
  });
}

int sisdc_profile_kernel(sisdc_handle* h, int kernel, int level, double dt_m, int reps, double* avg_us) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (reps < 1 || !avg_us) fail(SISDC_EINVAL, "reps >= 1 and an output pointer required");
    if (kernel < SISDC_K_SIPG_APPLY || kernel > SISDC_K_CG_UPDATE) fail(SISDC_EINVAL, "unknown kernel");
    hipStream_t s = h->stream;
    CoefP cf = coef_for(h, L, dt_m, L.um(0));
    const double* x = L.M >= 1 ? L.um(1) : L.um(0);
    // a CG state on the level's data: b = M u_1 + diag (never zero), x0 = 0,
    // never converging (rtol = 0)
    HIPCHECK(launch_helm_diag(L.diag, L.nv, cf, dt_m, h->ctau, L.g, L.tab, s));
    lincomb(h, L, L.b, {{1.0, x}, {1.0, L.diag}}, {1, 0});
    HIPCHECK(hipMemsetAsync(L.t2, 0, L.vlen * sizeof(double), s));
    const int id = ++h->solve_id;
    CGState cg = cg_state<double>(h, bufs64(h, L), L.b, L.t2, 0.0);
    // the kernels the PCG of this level runs (isotropic hexahedral path or general path)
    const bool iso = sipg_iso_path(L.g, cf);
    if (iso)
      HIPCHECK(launch_iso_inv_diag(L.diag, L.idg, cf, dt_m, h->ctau, L.g, L.tab, s));
    else
      HIPCHECK(launch_helm_diag(L.diag, L.nv, cf, dt_m, h->ctau, L.g, L.tab, s));
    HIPCHECK(launch_sipg(L.t2, L.cw, L.nv, cf, L.trace, 1.0, dt_m, h->ctau, L.g, L.tab, s));
    if (iso) {
      HIPCHECK(launch_cg_start_iso(cg, L.idg, L.nv, L.g, nullptr, L.mw, s));
      HIPCHECK(launch_sipg_apply_iso(L.cr, L.idg, L.cw, L.nv, cf, 1.0, dt_m, h->ctau, L.g, L.tab, cg.del,
                                     (const int*)nullptr, 0, s));
    } else {
      HIPCHECK(launch_cg_start(cg, L.nv, cf, L.g, L.tab, s));
      HIPCHECK(launch_sipg_apply(L.cz, L.cw, L.nv, cf, L.trace, 1.0, dt_m, h->ctau, L.g, L.tab, L.cz, cg.del,
                                 (const int*)nullptr, 0, s));
    }
    // CG update launches: one iteration 0 first, then iterations 1 and 2 in
    // turn (iteration 0 skips the p and s reads; the streaming form updates
    // x on odd iterations only), so the timed launches are representative
    int cg_it = 0;
    auto once = [&]() {
      switch (kernel) {
        case SISDC_K_SIPG_APPLY:
          if (iso)
            HIPCHECK(launch_sipg_apply_iso(L.cr, L.idg, L.t1, L.nv, cf, 1.0, dt_m, h->ctau, L.g, L.tab, cg.del,
                                           (const int*)h->done_gen, id, s));
          else
            HIPCHECK(launch_sipg_apply(L.cz, L.t1, L.nv, cf, L.trace, 1.0, dt_m, h->ctau, L.g, L.tab, L.cz, cg.del,
                                       (const int*)h->done_gen, id, s));
          break;
        case SISDC_K_SIPG_TRACE: HIPCHECK(launch_sipg_trace(L.cz, L.nv, cf, L.trace, L.g, L.tab, s)); break;
        case SISDC_K_CONV: conv(h, L, x, L.t1); break;
        default: {
          const int it = cg_it == 0 ? 0 : 1 + ((cg_it + 1) & 1);
          ++cg_it;
          if (iso)
            HIPCHECK(launch_cg_iter_iso(cg, L.idg, L.nv, L.g, it, id, s));
          else
            HIPCHECK(launch_cg_iter(cg, L.nv, cf, L.g, L.tab, it, id, s));
        }
      }
    };
    once();
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    HIPCHECK(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) once();
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_us = 1000.0 * ms / reps;
  });
}

int sisdc_net_init(sisdc_handle* h, int level, int hidden, unsigned long long seed, int max_batch, int max_rows) {
  return guard([&] {
    Level& L = level_at(h, level);
    if (hidden < 1 || max_batch < 1 || max_rows < 0) fail(SISDC_EINVAL, "hidden, max_batch >= 1, max_rows >= 0");
    net_free(L);
    auto& N = L.net;
    N.sh = MlpShape{L.np, hidden};
    N.max_batch = max_batch;
    N.max_rows = max_rows;
    const long P = N.sh.params();
    const int n = L.np, H = hidden;
    std::vector<float> th(P, 0.0f);
    // weights (2u - 1) sqrt(6 / fan_in), u from SplitMix64; biases 0
    long pos = 0;
    uint64_t k = 0;
    auto fill = [&](long cnt, int fan_in) {
      const double sc = std::sqrt(6.0 / fan_in);
      for (long i = 0; i < cnt; ++i) {
        const double u = (double)(splitmix64(seed, k++) >> 11) * (1.0 / 9007199254740992.0);
        th[pos + i] = (float)((2.0 * u - 1.0) * sc);
      }
      pos += cnt;
    };
    fill((long)H * n, n);
    pos += H;
    fill((long)H * H, H);
    pos += H;
    fill((long)n * H, H);
    N.theta = falloc(P);
    N.m = falloc(P);
    N.v = falloc(P);
    N.g = falloc(P);
    HIPCHECK(hipMemcpy(N.theta, th.data(), P * sizeof(float), hipMemcpyHostToDevice));
    HIPCHECK(hipMemset(N.m, 0, P * sizeof(float)));
    HIPCHECK(hipMemset(N.v, 0, P * sizeof(float)));
    const long B = max_batch, rows = (long)L.nv * L.E;
    N.Z1 = falloc(B * H);
    N.A1 = falloc(B * H);
    N.Z2 = falloc(B * H);
    N.A2 = falloc(B * H);
    N.Y = falloc(B * n);
    N.dY = falloc(B * n);
    N.dA = falloc(B * H);
    N.dZ = falloc(B * H);
    N.Xs = falloc(B * n);
    N.Ts = falloc(B * n);
    N.Xi = falloc(rows * n);
    N.A1i = falloc(rows * H);
    N.A2i = falloc(rows * H);
    N.Yi = falloc(rows * n);
    N.nrm = dalloc(rows);
    N.xnew = dalloc(L.vlen);
    N.x0h = dalloc(L.vlen);
    N.r0h = dalloc(L.vlen);
    N.Xd = falloc(std::max<long>(1, (long)max_rows * n));
    N.Td = falloc(std::max<long>(1, (long)max_rows * n));
    N.loss_cap = std::max(1, max_rows) + 1;
    N.lossp = dalloc((size_t)64 * N.loss_cap);
    N.on = true;
  });
}

int sisdc_net_get_params(sisdc_handle* h, int level, float* theta, int mem, long long* n) {
  return guard([&] {
    auto& N = net_of(h, level);
    if (n) *n = N.sh.params();
    if (!theta) return;
    HIPCHECK(hipMemcpyAsync(theta, N.theta, N.sh.params() * sizeof(float),
                            mem == SISDC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
  });
}

int sisdc_net_set_params(sisdc_handle* h, int level, const float* theta, int mem) {
  return guard([&] {
    auto& N = net_of(h, level);
    if (!theta) fail(SISDC_EINVAL, "null parameters");
    HIPCHECK(hipMemcpyAsync(N.theta, theta, N.sh.params() * sizeof(float),
                            mem == SISDC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
  });
}

int sisdc_net_forward(sisdc_handle* h, int level, const float* X, int rows, float* Y, int mem, int bf16) {
  return guard([&] {
    auto& N = net_of(h, level);
    if (!X || !Y || rows < 1 || rows > N.max_batch) fail(SISDC_EINVAL, "rows must be 1..max_batch");
    const long cnt = (long)rows * N.sh.n;
    const auto kin = mem == SISDC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const auto kout = mem == SISDC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIPCHECK(hipMemcpyAsync(N.Xs, X, cnt * sizeof(float), kin, h->stream));
    HIPCHECK(mlp_forward(N.sh, N.theta, N.Xs, rows, nullptr, N.A1, nullptr, N.A2, N.Y, bf16 ? 1 : 0, h->stream));
    HIPCHECK(hipMemcpyAsync(Y, N.Y, cnt * sizeof(float), kout, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
  });
}

int sisdc_net_train_step(sisdc_handle* h, int level, const float* X, const float* T, int rows, double lr, double* loss,
                         int mem) {
  return guard([&] {
    Level& L = level_at(h, level);
    auto& N = net_of(h, level);
    if (!X || !T || rows < 1 || rows > N.max_batch) fail(SISDC_EINVAL, "rows must be 1..max_batch");
    const long cnt = (long)rows * N.sh.n;
    const auto kin = mem == SISDC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIPCHECK(hipMemcpyAsync(N.Xs, X, cnt * sizeof(float), kin, h->stream));
    HIPCHECK(hipMemcpyAsync(N.Ts, T, cnt * sizeof(float), kin, h->stream));
    net_train_batch(h, L, N.Xs, N.Ts, rows, lr, N.lossp);
    std::vector<double> lp(64);
    HIPCHECK(hipMemcpyAsync(lp.data(), N.lossp, 64 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    double acc = 0.0;
    for (double v : lp) acc += v;
    if (loss) *loss = 0.5 * acc / rows;
  });
}

int sisdc_net_grad(sisdc_handle* h, int level, const float* X, const float* T, int rows, float* grad, double* loss,
                   int mem) {
  return guard([&] {
    auto& N = net_of(h, level);
    if (!X || !T || !grad || rows < 1 || rows > N.max_batch) fail(SISDC_EINVAL, "rows must be 1..max_batch");
    const long cnt = (long)rows * N.sh.n;
    const auto kin = mem == SISDC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const auto kout = mem == SISDC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    hipStream_t s = h->stream;
    HIPCHECK(hipMemcpyAsync(N.Xs, X, cnt * sizeof(float), kin, s));
    HIPCHECK(hipMemcpyAsync(N.Ts, T, cnt * sizeof(float), kin, s));
    HIPCHECK(mlp_forward(N.sh, N.theta, N.Xs, rows, N.Z1, N.A1, N.Z2, N.A2, N.Y, 0, s));
    HIPCHECK(mlp_backward(N.sh, N.theta, N.Xs, N.Ts, rows, N.Z1, N.A1, N.Z2, N.A2, N.Y, N.dY, N.dA, N.dZ, N.g,
                          N.lossp, s));
    HIPCHECK(hipMemcpyAsync(grad, N.g, N.sh.params() * sizeof(float), kout, s));
    std::vector<double> lp(64);
    HIPCHECK(hipMemcpyAsync(lp.data(), N.lossp, 64 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    double acc = 0.0;
    for (double v : lp) acc += v;
    if (loss) *loss = 0.5 * acc / rows;
  });
}

int sisdc_net_harvest(sisdc_handle* h, int level, int on, int* rows_out) {
  return guard([&] {
    auto& N = net_of(h, level);
    N.harvest = on != 0;
    if (on < 0) N.rows = 0;  // negative: clear the harvested rows
    if (rows_out) *rows_out = N.rows;
  });
}

int sisdc_net_train(sisdc_handle* h, int level, int epochs, int batch, double lr, double* loss) {
  return guard([&] {
    Level& L = level_at(h, level);
    auto& N = net_of(h, level);
    if (epochs < 1 || batch < 1 || batch > N.max_batch) fail(SISDC_EINVAL, "epochs >= 1, batch in 1..max_batch");
    if (N.rows < 1) fail(SISDC_ESTATE, "no harvested rows");
    const int nb = (N.rows + batch - 1) / batch;
    if (nb > N.loss_cap) fail(SISDC_EINVAL, "batch too small for the loss buffer");
    for (int ep = 0; ep < epochs; ++ep)
      for (int b = 0; b < nb; ++b) {
        const int r0 = b * batch, rows = std::min(batch, N.rows - r0);
        net_train_batch(h, L, N.Xd + (long)r0 * N.sh.n, N.Td + (long)r0 * N.sh.n, rows, lr, N.lossp + 64 * (long)b);
      }
    std::vector<double> lp((size_t)64 * nb);
    HIPCHECK(hipMemcpyAsync(lp.data(), N.lossp, lp.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    double acc = 0.0;
    for (double v : lp) acc += v;
    if (loss) *loss = 0.5 * acc / N.rows;  // mean loss of the last epoch
  });
}

int sisdc_net_use(sisdc_handle* h, int level, int on) {
  return guard([&] {
    auto& N = net_of(h, level);
    N.use = on != 0;
  });
}

// ------------------------------------------------------------------ batches
// Independent instances stepped together.  Every instance has its own handle
// and its own HIP stream, so the kernels of different instances overlap on
// the device; the host work (launches, the waits of the multi-kernel PCG and
// of the step's end) is spread over `threads` host threads, instance i on
// thread i mod threads.
}  // extern "C"

// With more than one host thread, each thread is a lane of the persistent-
// solve order: persistent solves small enough to share the device overlap
// those of the other threads, larger ones run alone.
struct sisdc_batch {
  std::vector<sisdc_handle*> h;
  std::vector<hipStream_t> streams;
  std::vector<int> variant;    // PCG form of each instance
  std::vector<int> precision;  // arithmetic of each instance's Helmholtz solves
  int threads = 1;
  int graph = 0;               // step graphs on every instance
};

namespace {

// f(i) for every instance on the batch's host threads; the first failing
// instance's code and message become the caller's.
template <class F>
int batch_run(sisdc_batch* b, F&& f) {
  const int n = (int)b->h.size();
  const int T = std::max(1, std::min(b->threads, n));
  std::vector<int> rc(n, SISDC_OK);
  std::vector<std::string> msg(n);
  auto work = [&](int t) {
    for (int i = t; i < n; i += T) {
      rc[i] = f(i);
      if (rc[i] != SISDC_OK) msg[i] = sisdc_last_error();
    }
  };
  if (T == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    pool.reserve(T);
    for (int t = 0; t < T; ++t) pool.emplace_back(work, t);
    for (auto& th : pool) th.join();
  }
  for (int i = 0; i < n; ++i)
    if (rc[i] != SISDC_OK) {
      g_last_error = "instance " + std::to_string(i) + ": " + msg[i];
      return rc[i];
    }
  g_last_error.clear();
  return SISDC_OK;
}

// Select the PCG form of every level of a handle (SISDC_CG_AUTO lets levels
// whose tiles fit use the persistent kernel).
void set_cg_variant(sisdc_handle* h, int variant) {
  h->meth.cg_variant = variant;
  for (auto& L : h->lv) L.persistent = persistent_fits(h, L, variant);
}

void set_form(sisdc_handle* h, int variant, int precision) {
  h->meth.precision = precision;
  set_cg_variant(h, variant);
}

}  // namespace

extern "C" {

int sisdc_batch_create(int n, const sisdc_problem* probs, const sisdc_method* meths, sisdc_batch** out) {
  if (!out) {
    g_last_error = "null output pointer";
    return SISDC_EINVAL;
  }
  *out = nullptr;
  if (n < 1 || !probs || !meths) {
    g_last_error = "n >= 1 and problem / method arrays required";
    return SISDC_EINVAL;
  }
  sisdc_batch* b = new (std::nothrow) sisdc_batch();
  if (!b) {
    g_last_error = "host allocation failed";
    return SISDC_ENOMEM;
  }
  for (int i = 0; i < n; ++i) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      sisdc_batch_destroy(b);
      g_last_error = "instance " + std::to_string(i) + ": hipStreamCreateWithFlags failed";
      return SISDC_EDEVICE;
    }
    b->streams.push_back(s);
    sisdc_handle* h = nullptr;
    const int rc = sisdc_create(&probs[i], &meths[i], (void*)s, &h);
    if (rc != SISDC_OK) {
      const std::string m = "instance " + std::to_string(i) + ": " + g_last_error;
      sisdc_batch_destroy(b);
      g_last_error = m;
      return rc;
    }
    b->h.push_back(h);
    b->variant.push_back(meths[i].cg_variant);
    b->precision.push_back(meths[i].precision);
  }
  b->threads = std::min(n, 8);
  *out = b;
  return SISDC_OK;
}

int sisdc_batch_destroy(sisdc_batch* b) {
  if (!b) return SISDC_OK;
  for (sisdc_handle* h : b->h) sisdc_destroy(h);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  delete b;
  return SISDC_OK;
}

int sisdc_batch_size(const sisdc_batch* b, int* n) {
  if (!b || !n) {
    g_last_error = "null batch or output pointer";
    return SISDC_EINVAL;
  }
  *n = (int)b->h.size();
  return SISDC_OK;
}

int sisdc_batch_handle(sisdc_batch* b, int i, sisdc_handle** h) {
  if (!b || !h || i < 0 || i >= (int)b->h.size()) {
    g_last_error = "null pointer or instance out of range";
    return SISDC_EINVAL;
  }
  *h = b->h[i];
  return SISDC_OK;
}

int sisdc_batch_set_threads(sisdc_batch* b, int threads) {
  if (!b || threads < 1 || threads > 64) {
    g_last_error = "threads in 1..64 required";
    return SISDC_EINVAL;
  }
  b->threads = threads;
  return SISDC_OK;
}

int sisdc_batch_set_graph(sisdc_batch* b, int on) {
  if (!b || (on != 0 && on != 1)) {
    g_last_error = "null batch or on not 0 / 1";
    return SISDC_EINVAL;
  }
  for (sisdc_handle* h : b->h) {
    const int rc = sisdc_set_graph(h, on);
    if (rc != SISDC_OK) return rc;
  }
  b->graph = on;
  return SISDC_OK;
}

int sisdc_batch_step(sisdc_batch* b, const double* dt, sisdc_stats* st) {
  if (!b || !dt) {
    g_last_error = "null batch or dt";
    return SISDC_EINVAL;
  }
  const int n = (int)b->h.size();
  const int T = std::max(1, std::min(b->threads, n));  // as in batch_run: instance i on thread i mod T
  for (int i = 0; i < n; ++i) {
    set_form(b->h[i], b->variant[i], b->precision[i]);
    b->h[i]->lane = T > 1 ? i % T : -1;
    b->h[i]->lanes = T;
  }
  const int rc = batch_run(b, [&](int i) { return sisdc_step(b->h[i], 0.0, dt[i], st ? &st[i] : nullptr); });
  for (sisdc_handle* h : b->h) h->lane = -1;
  return rc;
}

// Autotuner: per instance, the form of its Helmholtz solves (persistent PCG
// where it fits, or multi-kernel; for an instance configured for mixed
// precision also plain FP64, which meets the same FP64 residual tolerance),
// then the number of host threads for the whole batch, each by the wall
// time of one step from the same state, which is restored afterwards.
int sisdc_batch_tune(sisdc_batch* b, const double* dt, int* threads_out, int* variants_out, int* precisions_out,
                     int* graph_out) {
  if (!b || !dt) {
    g_last_error = "null batch or dt";
    return SISDC_EINVAL;
  }
  const int n = (int)b->h.size();
  std::vector<double*> saved(n, nullptr);
  auto release = [&]() {
    for (double* p : saved)
      if (p) (void)hipFree(p);
  };
  for (int i = 0; i < n; ++i) {
    sisdc_handle* h = b->h[i];
    if (!h->have_state) {
      release();
      g_last_error = "instance " + std::to_string(i) + ": sisdc_set_state must precede sisdc_batch_tune";
      return SISDC_ESTATE;
    }
    if (hipMalloc(&saved[i], h->lv[0].vlen * sizeof(double)) != hipSuccess) {
      release();
      g_last_error = "hipMalloc failed";
      return SISDC_ENOMEM;
    }
    if (hipMemcpyAsync(saved[i], h->state, h->lv[0].vlen * sizeof(double), hipMemcpyDeviceToDevice, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      release();
      g_last_error = "state copy failed";
      return SISDC_EDEVICE;
    }
  }
  auto restore = [&](int i) { return sisdc_set_state(b->h[i], saved[i], SISDC_MEM_DEVICE); };
  for (sisdc_handle* h : b->h) h->graph_on = false;  // instances are timed uncaptured first
  auto now = []() { return std::chrono::steady_clock::now(); };
  auto secs = [](auto a, auto c) { return std::chrono::duration<double>(c - a).count(); };
  int rc = SISDC_OK;
  for (int i = 0; i < n && rc == SISDC_OK; ++i) {
    sisdc_handle* h = b->h[i];
    h->lane = -1;
    const int configured = b->precision[i];
    std::vector<std::pair<int, int>> forms = {{SISDC_CG_AUTO, configured}, {SISDC_CG_MULTI_KERNEL, configured}};
    if (configured == SISDC_MIXED) {
      forms.emplace_back(SISDC_CG_AUTO, SISDC_FP64);
      forms.emplace_back(SISDC_CG_MULTI_KERNEL, SISDC_FP64);
    }
    double best = 1e300;
    std::pair<int, int> pick = forms[0];
    for (const auto& f : forms) {
      set_form(h, f.first, f.second);
      if ((rc = sisdc_step(h, 0.0, dt[i], nullptr)) != SISDC_OK) break;  // warm-up of this form
      if ((rc = restore(i)) != SISDC_OK) break;
      const auto t0 = now();
      if ((rc = sisdc_step(h, 0.0, dt[i], nullptr)) != SISDC_OK) break;
      const double tv = secs(t0, now());
      if ((rc = restore(i)) != SISDC_OK) break;
      if (tv < best) {
        best = tv;
        pick = f;
      }
    }
    set_form(h, pick.first, pick.second);
    b->variant[i] = pick.first;
    b->precision[i] = pick.second;
    if (variants_out) variants_out[i] = pick.first;
    if (precisions_out) precisions_out[i] = pick.second;
  }
  const int graph_before = b->graph;
  double best_steps = 1e300;
  if (rc == SISDC_OK) rc = sisdc_batch_set_graph(b, 0);
  if (rc == SISDC_OK) {
    int pick = b->threads;
    for (int T : {1, 2, 4, 8, 16}) {
      if (T > n && T != 1) continue;
      b->threads = T;
      const auto t0 = now();
      if ((rc = sisdc_batch_step(b, dt, nullptr)) != SISDC_OK) break;
      const double tv = secs(t0, now());
      for (int i = 0; i < n && rc == SISDC_OK; ++i) rc = restore(i);
      if (rc != SISDC_OK) break;
      if (tv < best_steps) {
        best_steps = tv;
        pick = T;
      }
    }
    b->threads = pick;
    if (threads_out) *threads_out = pick;
  }
  if (rc == SISDC_OK) {  // step graphs: one step captures, the next is timed
    int pick = 0;
    if ((rc = sisdc_batch_set_graph(b, 1)) == SISDC_OK && (rc = sisdc_batch_step(b, dt, nullptr)) == SISDC_OK) {
      for (int i = 0; i < n && rc == SISDC_OK; ++i) rc = restore(i);
      const auto t0 = now();
      if (rc == SISDC_OK && (rc = sisdc_batch_step(b, dt, nullptr)) == SISDC_OK) {
        const double tv = secs(t0, now());
        for (int i = 0; i < n && rc == SISDC_OK; ++i) rc = restore(i);
        if (tv < best_steps) pick = 1;
      }
    }
    if (rc == SISDC_OK) rc = sisdc_batch_set_graph(b, pick);
    if (graph_out) *graph_out = pick;
  } else {
    (void)sisdc_batch_set_graph(b, graph_before);
  }
  const std::string m = g_last_error;
  release();
  g_last_error = rc == SISDC_OK ? std::string() : m;
  return rc;
}

}  // extern "C"
