/*
 * sisdc.h -- C ABI of libsisdc: semi-implicit (multilevel) spectral deferred
 * correction, SI-SDC / SI-MLSDC, with a nodal DG-SEM discretisation on
 * periodic Cartesian meshes, running on AMD MI355X (gfx950).
 *
 * Method: Pfister & Stiller, "Semi-implicit multilevel spectral deferred
 * correction" (arXiv 2504.18526).
 *   - problem:  u_t + div f_c(u) = div f_d(u, grad u)              (Sec. 2)
 *   - SDC:      incremental collocation on M Radau-right nodes, SI(1)/SI(2)
 *               predictor and corrector                            (Sec. 3)
 *   - MLSDC:    FAS right-hand side, transfers I, P, R = I^T, V-cycle,
 *               cascade and FMG starts                 (Sec. 4, Alg. 1-4)
 *   - space:    DG on piecewise polynomials of degree P per element (Sec. 6)
 *
 * Conventions shared by every call
 *   Errors     every call returns int: SISDC_OK (0) or a negative code below;
 *              sisdc_last_error() returns a message for the calling thread.
 *              No C++ exception or abort crosses the ABI.  SISDC_ENOTCONV
 *              still leaves the best iterate in the output.
 *   Memory     `mem` says whether the caller's pointers are host memory
 *              (SISDC_MEM_HOST) or device memory of the handle's GPU
 *              (SISDC_MEM_DEVICE).  Caller buffers are only read/written
 *              during the call; the library keeps no caller pointer.  The
 *              handle owns every level and work buffer.
 *   Streams    the handle is bound to one hipStream_t at creation (NULL: the
 *              null stream); every call is stream-ordered and returns after
 *              its work has completed (calls synchronise the stream).  The
 *              library accesses caller device buffers on the handle's
 *              stream: work on other streams that produces an input (or
 *              still uses an output buffer) must be complete before the
 *              call.
 *   Threads    one handle is used by one thread at a time.
 *   Levels     level index 0 is the FINEST level, n_levels-1 the coarsest
 *              (the paper numbers levels the other way, l = 1 coarsest).
 *   Layout     a nodal vector is double u[var][elem][node]: elem =
 *              e_x + n_x (e_y + n_y e_z) (x fastest), node = i_x + (P+1)
 *              (i_y + (P+1) i_z) on the Gauss-Lobatto-Legendre points, x
 *              fastest.  Collocation arrays are [m][var][elem][node] with
 *              m = 0..M, m = 0 being the step's initial value u_0.
 *   Weak form  right-hand sides, residuals and FAS terms g live in the dual
 *              space: the value at a node is the functional tested with that
 *              node's basis function (the discrete collocation equation of
 *              Sec. 6 is written this way).  Mass matrix: GLL-lumped.
 */
#ifndef SISDC_H
#define SISDC_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SISDC_OK = 0,
  SISDC_EINVAL = -1,     /* invalid argument (message says which)          */
  SISDC_ENOMEM = -2,     /* device or host allocation failed               */
  SISDC_EDEVICE = -3,    /* a HIP runtime call failed                      */
  SISDC_ENOTCONV = -4,   /* an implicit solve missed its tolerance         */
  SISDC_ENONFINITE = -5, /* a non-finite value appeared in the state       */
  SISDC_ESTATE = -6      /* call order violated (e.g. step before state)   */
};

enum { SISDC_MEM_HOST = 0, SISDC_MEM_DEVICE = 1 };

typedef enum {
  SISDC_EQ_CONVDIFF = 0, /* u_t + div(a u) = nu lap u           (Sec. 2)   */
  SISDC_EQ_BURGERS = 1,  /* u_t + div(u^2/2 (1,..,1)) = nu lap u (Sec. 2)  */
  SISDC_EQ_EULER = 2,    /* compressible Euler, perfect gas      (Sec. 2)  */
  SISDC_EQ_NS = 3        /* compressible Navier-Stokes, constant mu, Pr;
                            viscous term by BR1 lifting          (Sec. 2)  */
} sisdc_eq;

enum { SISDC_SI2 = 0, SISDC_SI1 = 1, SISDC_IMEX_EULER = 2 };  /* Sec. 3 */
enum { SISDC_PROJ_INTERP = 0, SISDC_PROJ_L2 = 1 };                /* Sec. 4 */
enum { SISDC_INCREMENTAL = 0, SISDC_NONINCREMENTAL = 1 };        /* Sec. 3, 4 */
enum { SISDC_NODES_RADAU_RIGHT = 0, SISDC_NODES_LOBATTO = 1 };  /* Sec. 3 */
enum { SISDC_START_CASCADE = 0, SISDC_START_FMG = 1,   /* Alg. 3, Alg. 4    */
       SISDC_START_PREDICTOR = 2,                      /* Sec. 4: the SI
                                                          predictor on every
                                                          level              */
       SISDC_START_CONSTANT = 3 };                     /* Sec. 4: u_0 spread
                                                          to every node of
                                                          every level        */
enum { SISDC_FP64 = 0,   /* every solve in FP64                             */
       SISDC_MIXED = 1 }; /* FP32 Jacobi-PCG inside FP64 iterative refinement:
                             the outer residual b - A x, the solution update,
                             the node quadrature and the node updates stay
                             FP64; operators and CG vectors of the inner
                             solves are FP32 with FP32 accumulation        */
enum { SISDC_CG_AUTO = 0, SISDC_CG_MULTI_KERNEL = 1, SISDC_CG_PERSISTENT_COOPERATIVE = 2 };
enum { SISDC_PRECOND_JACOBI = 0,  /* point Jacobi (the diagonal of A)               */
       SISDC_PRECOND_FDS = 1 };   /* element-block Jacobi by fast diagonalisation
                                     (Sec. 8, "Runtime analysis": the paper's
                                     alternative to PCG, here as a preconditioner) */

typedef struct {
  int dim;             /* 2 or 3                                            */
  int n_elem[3];       /* elements per axis (periodic uniform mesh)         */
  double lo[3], hi[3]; /* box                                               */
  int eq;              /* sisdc_eq                                          */
  double a[3];         /* convection velocity (CONVDIFF)                    */
  double nu;           /* diffusivity (CONVDIFF, BURGERS)                   */
  double gamma;        /* ratio of specific heats (EULER, NS)               */
  double mu;           /* dynamic viscosity (NS)                            */
  double Pr;           /* Prandtl number (NS)                               */
  double R;            /* gas constant (EULER, NS; <= 0 means 1)            */
  int stack;           /* 0 or 1: one instance.  B > 1: an ensemble of B
                          independent instances of this problem stacked
                          along the last axis, each on its own periodic box
                          of n_elem elements: the handle's state holds B
                          consecutive element blocks (instance k: elements
                          k E .. (k+1) E - 1 of every component, E the
                          elements of one instance) and every kernel of a
                          step runs once for all of them.  The instances
                          share dt, the method and each Helmholtz solve:
                          their systems are solved as one block-diagonal
                          system, stopped on the joint relative residual.
                          Scalar equations only (CONVDIFF, BURGERS), with
                          conserve = 0 (the conservation shift is one
                          constant per component) and no h_coarsen          */
} sisdc_problem;

typedef struct {
  int n_levels;        /* 1..3                                              */
  int P[3];            /* polynomial degree per level (index 0 finest), 1..8 */
  int M[3];            /* collocation nodes per level, 1..8 (see nodes)    */
  int integrator;      /* SISDC_SI2 (default), SISDC_SI1, or SISDC_IMEX_EULER
                          (eq. H_IMEX: the one-stage form with the physical
                          diffusion alone implicit, nu I for the scalar
                          equations; systems keep no implicit term, their
                          substeps are explicit apart from the mass matrix) */
  int start;           /* SISDC_START_*  (multilevel only)                  */
  int n_coarse_sweeps; /* N_c, sweeps on the coarsest level per V-cycle     */
  int post_sweep;      /* final fine sweep after the last V-cycle (0/1)     */
  int n_iter;          /* sweeps K (one level) or V-cycles C (multilevel)   */
  double cg_rtol;      /* relative residual ||b-Ax||_2 <= rtol ||b||_2      */
  int cg_maxit;        /* iteration cap per solve                           */
  double c_tau;        /* SIPG penalty factor C_tau (tau = C_tau (P+1)^2 kappa / h) */
  int precision;       /* SISDC_FP64 or SISDC_MIXED                         */
  int cg_variant;      /* SISDC_CG_AUTO: one persistent launch per solve
                          (pipelined PCG) for scalar equations when the
                          level's elements fit on the GPU at once and
                          rtol >= 1e-11, else the multi-kernel form.  The
                          persistent kernel is an ordinary launch whose
                          grid fits the device at once; the library orders
                          its persistent solves across streams and handles
                          (each waits for the previous one, wherever it
                          ran), so two never share the device.  Kernels of
                          other code that wait on each other across
                          workgroups must not run at the same time;
                          SISDC_CG_MULTI_KERNEL: always the multi-kernel
                          form;
                          SISDC_CG_PERSISTENT_COOPERATIVE: as AUTO, but the
                          persistent kernel goes through the cooperative-
                          launch API, which checks co-residency itself and
                          costs about 25 us more per solve (the queue hand-
                          over before and after the kernel)               */
  double inner_rtol;   /* SISDC_MIXED: relative tolerance of each FP32 inner
                          solve (<= 0: 1e-5)                                */
  int projection;      /* P_x, the fine-to-coarse solution transfer (Sec. 4,
                          "MLSDC transfer operators"): SISDC_PROJ_INTERP
                          (embedded interpolation, default) or SISDC_PROJ_L2
                          (L^2 projection onto each element's coarse
                          polynomials, (I^T W_f I)^-1 I^T W_f per axis)     */
  int formulation;     /* SISDC_INCREMENTAL (node-to-node, default) or
                          SISDC_NONINCREMENTAL (zero-to-node, Sec. 4
                          "Non-incremental multilevel SDC method"): equal
                          on one level; with several levels the FAS terms
                          and residuals are node sums, so the residual
                          restriction in time becomes C_c^-1 I_t^T C_f    */
  int nodes;           /* collocation nodes in time (Sec. 3): SISDC_NODES_
                          RADAU_RIGHT (default; Radau IIA, order 2M - 1) or
                          SISDC_NODES_LOBATTO (both end points, tau_1 = 0 so
                          u_1 = u_0; Lobatto IIIA, order 2M - 2; M >= 2)    */
  int h_coarsen[3];    /* 1: level l has half the elements of level l - 1
                          along every axis (2:1 h-coarsening, Sec. 6
                          "MLSDC transfer operators"; the counts must be
                          even; in 3-D the finer degree must be <= 6);
                          h_coarsen[0] = 0                                   */
  int c_fmg;           /* SISDC_START_FMG: V-cycles per added level, C_fmg of
                          Alg. 4 (FMG_1, FMG_2, ...); <= 0 means 1.  With two
                          levels the FMG start equals the cascade start    */
  int conserve;        /* 1: after every implicit solve each component of the
                          solution is shifted by the constant that makes its
                          total 1^T M x equal the right-hand side's total (the
                          exact solution has it, since the SIPG operator is
                          symmetric with the constants in its kernel), so the
                          totals the method conserves hold to round-off at any
                          PCG tolerance; 0: the iterate as the PCG leaves it
                          (totals drift by up to the tolerance per solve)   */
  int precond;         /* PCG preconditioner: SISDC_PRECOND_JACOBI (default)
                          or SISDC_PRECOND_FDS: on levels whose implicit
                          coefficient is isotropic and constant (the systems'
                          kappa_m I; the scalar equations under IMEX Euler),
                          z = A_ee^-1 r per element, A_ee the element's
                          diagonal block of M + dt_m K, applied exactly by
                          fast diagonalisation (one small eigenproblem per
                          axis at set-up); FP64 solves of those levels only,
                          other levels and the FP32 inner solves keep Jacobi */
  double av_kappa;     /* kappa_s and c_s of the Persson-Peraire artificial */
  double av_c;         /* viscosity (Sec. 6: the diffusion matrix supplemented
                          for shocks; Sec. 8 gives kappa_s, c_s per test).
                          av_c > 0 switches it
                          on: at the start of every step, from u_0 on the
                          finest level, per element e the share S_e of the
                          L2 energy of u (the density of a system) in the
                          Legendre modes of degree P, s_e = log10 S_e,
                          s_0 = -4 log10 P, and
                            eps_e = eps_0 sw((s_e - s_0) / kappa_s),
                            sw(r) = 0 (r < -1), 1 (r > 1),
                                    (1 + sin(pi r / 2)) / 2 between,
                            eps_0 = c_s (min_d h_d / P) lam_e,
                          lam_e the largest wave speed over the element's
                          nodes; eps_e grad u joins the diffusive flux of
                          every component (in F and in the implicit
                          coefficient D_m) for the whole step, on every
                          level.  Requires the same elements on every level
                          (no h_coarsen) and FP64 solves (precision
                          SISDC_FP64) and av_kappa > 0; the levels take the
                          multi-kernel PCG                                  */
} sisdc_method;

typedef struct {
  int fine_sweeps;        /* predictor + corrector sweeps on level 0        */
  int solves;             /* Helmholtz solves on all levels                 */
  long long cg_iters;     /* CG iterations summed over all solves           */
  int cg_iters_max;       /* largest iteration count of one solve           */
  int not_converged;      /* solves that hit cg_maxit                       */
  double max_rel_residual;/* largest final relative residual                */
  int ir_rounds;          /* SISDC_MIXED: FP32 inner solves (refinement rounds) */
  int net_guesses;        /* learned initial guesses computed               */
  int net_rejected;       /* ... of which refused (no positive step)        */
  int ir_fallbacks;       /* SISDC_MIXED: solves whose refinement stalled (a
                             round that did not halve the FP64 residual, or
                             20 rounds) and that FP64 PCG finished          */
} sisdc_stats;

typedef struct {
  int iters;
  int converged;
  double rel_residual;
} sisdc_solve_stats;

typedef struct sisdc_handle sisdc_handle;

/* Thread-local message of the last failing call ("" if none). */
const char* sisdc_last_error(void);

/* Create a handle for `prob` discretised with `meth` on the current HIP
 * device, bound to `hip_stream` (a hipStream_t, NULL = null stream).
 * Validates every field (EINVAL), allocates all level buffers (ENOMEM). */
int sisdc_create(const sisdc_problem* prob, const sisdc_method* meth,
                 void* hip_stream, sisdc_handle** out);
int sisdc_destroy(sisdc_handle* h);

/* Sizes of a level: elements, nodes per element, variables, M. */
int sisdc_level_info(const sisdc_handle* h, int level, int* n_elem_total,
                     int* nodes_per_elem, int* n_var, int* M);

/* Physical node coordinates of a level, x[d][elem][node] (d < dim). */
int sisdc_node_coords(sisdc_handle* h, int level, double* x, int mem);

/* Fine-level initial value u_0 (one nodal vector, [var][elem][node]). */
int sisdc_set_state(sisdc_handle* h, const double* u0, int mem);

/* Read / write the collocation iterate of a level, all nodes m = 0..M
 * ([m][var][elem][node]).  Writing it also marks the stored f, C and
 * K-terms of that level stale (they are recomputed on the next sweep). */
int sisdc_get_level(sisdc_handle* h, int level, double* u, int mem);
int sisdc_set_level(sisdc_handle* h, int level, const double* u, int mem);

/* Read / write the FAS right-hand side g of a level ([m-1][var][elem][node],
 * m = 1..M, weak form).  Level 0 normally has g = 0 (eq. ml-cm fas-mg rhs). */
int sisdc_get_fas(sisdc_handle* h, int level, double* g, int mem);
int sisdc_set_fas(sisdc_handle* h, int level, const double* g, int mem);

/* The fine solution at t+dt (u_{M}) after the last sisdc_step. */
int sisdc_get_state(sisdc_handle* h, double* u, int mem);

/* Per-step parameter of the systems' implicit term kappa_m I: lam* = max
 * over the nodes of max_d(|v_d| + c) of the current fine u_0 (EULER, NS; 0
 * otherwise), and for NS rho_min; kappa_m = (dt_m/2) lam*^2 (+ max(4 mu /
 * (3 rho_min), gamma mu / (Pr rho_min)) for NS).  Computed on the device at
 * the start of every step; this call computes it from the current fine u_0
 * and stores it for the next sweeps. */
int sisdc_update_step_params(sisdc_handle* h, double* lam_out);

/* One time step of length dt from the stored fine u_0 (Sec. 3 and 4):
 * one level: SI predictor and n_iter corrector sweeps; several levels:
 * start strategy (Alg. 3 / Alg. 4), n_iter V-cycles (Alg. 2) and an
 * optional fine post-sweep.  Afterwards u_0 <- u_{fine, M}. */
int sisdc_step(sisdc_handle* h, double t, double dt, sisdc_stats* st);

/* SI predictor on a level from that level's u_0 (eqs. sdc incremental
 * predictor si1/si2): fills u_1..u_M. */
int sisdc_predict(sisdc_handle* h, int level, double dt, sisdc_stats* st);

/* One incremental SI corrector sweep on a level (Alg. 1, N = 1, eqs.
 * sdc incremental corrector / DeltaH_SI1 / DeltaH_SI2 / ml-sdc incremental).
 * g: FAS right-hand side ([m-1][var][elem][node]); NULL uses the level's
 * stored g (zero unless set by a V-cycle or sisdc_set_fas). */
int sisdc_sweep(sisdc_handle* h, int level, double dt, const double* g, int mem,
                sisdc_stats* st);

/* One MLSDC V-cycle (Alg. 2) on levels top_level (finest of the cycle)
 * down to the coarsest, g = 0 on top_level. */
int mlsdc_vcycle(sisdc_handle* h, int top_level, double dt, sisdc_stats* st);

/* Solve (M + dt_m K_D) x = b on a level (the implicit part of H^SI, eq.
 * H_SI(1)) by Jacobi-preconditioned CG: on entry x holds the initial guess,
 * on exit the solution.  coef_state: u_b, the state the coefficient D is
 * evaluated at (BURGERS needs it; may be NULL otherwise).  b, x, coef_state
 * are nodal vectors ([var][elem][node]).  rtol <= 0 / maxit <= 0 select the
 * handle's cg_rtol / cg_maxit. */
int helmholtz_solve(sisdc_handle* h, int level, double dt_m, const double* coef_state,
                    const double* b, double* x, int mem, double rtol, int maxit,
                    sisdc_solve_stats* st);

/* helmholtz_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same solve, with the multi-kernel Jacobi-PCG in FP64 (no
 * learned guess, no mixed precision), whose work vectors, partial sums and
 * convergence record live in a fixed scratch array of 32 MiB that each GPU
 * holds until the process ends.  b, x and coef_state are device pointers of
 * the handle's GPU, which must be the current device.  The call allocates
 * nothing (its first call on a GPU only looks up the array's address).
 * Levels whose work space exceeds the array (about 6 level vectors plus face
 * traces: about 600 000 values per vector at most) are rejected with
 * SISDC_EINVAL.
 * Calls on one GPU share the array: calls that overlap on one GPU (other
 * handles, other streams, other threads) race.  The call synchronises the
 * handle's stream before it returns. */
int helmholtz_solve_noalloc(sisdc_handle* h, int level, double dt_m, const double* coef_state, const double* b,
                            double* x, double rtol, int maxit, sisdc_solve_stats* st);

/* Stage-level entry points (one operator application each, for parity
 * checks and for callers that compose their own schemes):
 *   SISDC_OP_MASS    out = M in
 *   SISDC_OP_CONV    out = C(in)                 weak convective operator
 *   SISDC_OP_FRHS    out = F(in) = C(in) - K_nu in (scalars), C(in) (Euler)
 *   SISDC_OP_SIPG    out = K_D in, D = D_m(aux) at step dt_m (aux may be NULL)
 *   SISDC_OP_HELM    out = M in + dt_m K_D in
 *   SISDC_OP_PROJECT out(level+1) = P_x in(level)       (space, fine->coarse)
 *   SISDC_OP_INTERP  out(level)   = I_x in(level+1)     (space, coarse->fine)
 *   SISDC_OP_RESTRICT out(level+1) = I_x^T in(level)    (space, fine->coarse)
 *   SISDC_OP_QUAD    out[m] = sum_i S_{m,i} in[i], S = dt_m w^nn (eq.
 *                    nn_weights; dt_m here is the step dt): in and out hold
 *                    M nodal vectors each ([m][var][elem][node], nodes 1..M)
 *   SISDC_OP_PRECOND out = A_ee^-1 in per element: the element-block Jacobi
 *                    preconditioner of M + dt_m K_D (isotropic constant D
 *                    only, else SISDC_EINVAL), by fast diagonalisation
 * All other vectors are single nodal vectors of the named level. */
enum { SISDC_OP_MASS = 0, SISDC_OP_CONV = 1, SISDC_OP_FRHS = 2, SISDC_OP_SIPG = 3,
       SISDC_OP_HELM = 4, SISDC_OP_PROJECT = 5, SISDC_OP_INTERP = 6,
       SISDC_OP_RESTRICT = 7, SISDC_OP_QUAD = 8, SISDC_OP_PRECOND = 9 };
int sisdc_apply(sisdc_handle* h, int op, int level, double dt_m, const double* in,
                const double* aux, double* out, int mem);

/* Collocation residual F_l(u) of a level's stored iterate, eq. cm
 * incremental op in weak form: out[m-1] = M (u_m - u_{m-1}) - q_m(u). */
int sisdc_collocation_residual(sisdc_handle* h, int level, double dt, double* out, int mem);

/* Measurement hook: average device time (microseconds) of one launch of a
 * hot-path kernel on a level, from HIP events recorded on the handle's stream
 * around `reps` back-to-back launches.  Inputs are the level's current
 * iterate (u_1, with the coefficient state u_0) at step dt_m; only scratch
 * vectors of the handle are written.  kernel:
 *   SISDC_K_SIPG_APPLY  the CG matvec pass M x + dt_m K_D x with its fused
 *                       dot product (face traces from SISDC_K_SIPG_TRACE)
 *   SISDC_K_SIPG_TRACE  the face-flux trace pass of the SIPG operator
 *   SISDC_K_CONV        the convective operator C(u)
 *   SISDC_K_CG_UPDATE   the CG vector update with its two dot products
 *                       (iteration 0 once, then iterations 1 and 2 in turn)
 * On isotropic levels (the systems' kappa_m I) the matvec and the update are
 * those of the streaming PCG: the matvec forms z = r / diag itself and
 * computes the neighbours' face fluxes (no trace pass). */
enum { SISDC_K_SIPG_APPLY = 0, SISDC_K_SIPG_TRACE = 1, SISDC_K_CONV = 2, SISDC_K_CG_UPDATE = 3 };
int sisdc_profile_kernel(sisdc_handle* h, int kernel, int level, double dt_m, int reps, double* avg_us);

/* Measurement hook for the persistent PCG (one cooperative launch per
 * Helmholtz solve, used for levels whose tiles are co-resident and for
 * tolerances >= 1e-11).  With on >= 1 the handle records a pair of HIP events
 * on its stream around every persistent launch and accumulates, per level,
 * the launches, the CG iterations they report and the event time between
 * each pair; switching on clears the sums.  on = 0 stops recording (the sums
 * are kept).  Results of launches still in flight are collected first, so
 * both calls synchronise the handle's stream. */
int sisdc_pcg_timing(sisdc_handle* h, int on);
/* The sums of sisdc_pcg_timing for one level: launches, iterations and total
 * event time in microseconds (any output pointer may be NULL). */
int sisdc_pcg_timing_get(sisdc_handle* h, int level, long long* launches, long long* iters,
                         double* total_us);
/* The same switch also times the multi-kernel PCG (the Chronopoulos-Gear
 * form of Sec. 8's implicit solves, used for systems, large levels and
 * tolerances below 1e-11): while it is on, in every on-th multi-kernel solve
 * of the handle (on = 1: every solve) a HIP event is recorded on the
 * handle's stream before and after every vector-update launch and after
 * every matvec launch, and the elapsed times of the launches that did a full
 * iteration's work (not the one that only found convergence, nor those that
 * exit at once behind it) are summed per level.  kernel: SISDC_K_CG_UPDATE
 * (the vector update with its two dot products) or SISDC_K_SIPG_APPLY (the
 * matvec with its dot product).  Launches of FP32 inner solves (SISDC_MIXED)
 * count as well.  Each event costs several microseconds of queue work, so a
 * stride above 1 keeps the timed run close to the untimed one. */
int sisdc_cg_kernel_timing_get(sisdc_handle* h, int level, int kernel, long long* launches, double* total_us);

/* Artificial viscosity (method av_c > 0): sisdc_av_update evaluates eps_e
 * from the current state (sisdc_set_state) as a step does from u_0, for
 * the operator hooks (sisdc_apply), which use the eps last evaluated (by a
 * step or by this call); sisdc_av_get copies eps_e (E_fine doubles, element
 * order x fastest) to host or device memory.  Both fail with SISDC_EINVAL on
 * a handle without it. */
int sisdc_av_update(sisdc_handle* h);
int sisdc_av_get(sisdc_handle* h, double* eps, int mem);

/* Step graphs (the launch side of the time step, Sec. 4's sweeps as one unit
 * of device work).  With on = 1, sisdc_step captures the whole step into a
 * HIP graph the first time and replays it afterwards: one graph launch per
 * step instead of one launch per kernel, and the host waits once, at the end
 * of the step, to collect the solves' result records.  A step can be
 * captured when every Helmholtz solve of it is a persistent PCG launch (a
 * scalar equation, FP64 solves, every level within the persistent kernel's
 * limits, tolerance >= 1e-11, no learned guess, PCG timing off); every solve
 * still stops on its own convergence test on the device, so a replayed step
 * gives the same result as the uncaptured step, bit for bit.  The graph
 * holds the step size and the solver form: a step with another dt, or after
 * the form changed, captures again.  A step that cannot be captured runs as
 * usual (uncaptured).  on = 0 releases the graph. */
int sisdc_set_graph(sisdc_handle* h, int on);
/* Graph counters: whether the last sisdc_step ran through the graph, and the
 * captures and graph launches so far (any output pointer may be NULL). */
int sisdc_graph_info(sisdc_handle* h, int* last_step_graphed, long long* captures, long long* replays);

/* Learned initial guess of a level's Helmholtz solves: an element-local MLP
 * n -> H -> H -> n (n = (P+1)^d, ReLU) applied to every (element, component)
 * row of the mass-scaled initial residual z0 = M^-1 (b - A x0), normalised to
 * unit norm; its output, times |z0_row|, is a correction delta, and x0
 * moves along it by the step that minimises the A-norm of the error,
 * alpha = (delta, r0) / (delta, A delta) (decided on the device; a step that
 * is not positive is refused and counted in the stats).  PCG always follows
 * to the same tolerance, so the network changes the initial guess only, and
 * never raises the error's A-norm.  Not part of the paper's method.
 *   sisdc_net_init     allocate; weights (2u - 1) sqrt(6 / fan_in) with u from
 *                      SplitMix64(seed) in parameter order, biases 0; Adam
 *                      state zero.  max_batch bounds training batches and
 *                      forward calls, max_rows the harvested rows.
 *   sisdc_net_get_params / set_params   flat FP32 parameters: W1 (H x n), b1,
 *                      W2 (H x H), b2, W3 (n x H), b3, row-major [out][in].
 *   sisdc_net_forward  y = N(x) for `rows` rows; bf16 != 0 rounds weights and
 *                      layer inputs to bfloat16 (nearest even), FP32 accumulate.
 *   sisdc_net_train_step  one Adam step (lr, beta 0.9 / 0.999, eps 1e-8) on the
 *                      loss 1/(2 rows) sum |N(x) - t|^2 in FP32; returns it.
 *   sisdc_net_grad     the same loss and its gradient (flat layout), no update.
 *   sisdc_net_harvest  on = 1: every later solve of the level appends rows
 *                      (z0 / |z0|, (x* - x0) / |z0|) until max_rows; 0: stop;
 *                      -1: stop and clear.  rows_out: rows held.
 *   sisdc_net_train    epochs over the harvested rows in order, batches of
 *                      `batch`; loss: mean loss of the last epoch.
 *   sisdc_net_use      on = 1: apply the network before every solve.   */
int sisdc_net_init(sisdc_handle* h, int level, int hidden, unsigned long long seed, int max_batch, int max_rows);
int sisdc_net_get_params(sisdc_handle* h, int level, float* theta, int mem, long long* n_params);
int sisdc_net_set_params(sisdc_handle* h, int level, const float* theta, int mem);
int sisdc_net_forward(sisdc_handle* h, int level, const float* x, int rows, float* y, int mem, int bf16);
int sisdc_net_train_step(sisdc_handle* h, int level, const float* x, const float* t, int rows, double lr,
                         double* loss, int mem);
int sisdc_net_grad(sisdc_handle* h, int level, const float* x, const float* t, int rows, float* grad,
                   double* loss, int mem);
int sisdc_net_harvest(sisdc_handle* h, int level, int on, int* rows_out);
int sisdc_net_train(sisdc_handle* h, int level, int epochs, int batch, double lr, double* loss);
int sisdc_net_use(sisdc_handle* h, int level, int on);

/* ---- Batches of independent instances ----
 * n instances (problem i, method i), each with its own handle and its own
 * HIP stream created by the batch, so the kernels of different instances
 * overlap on the device.  The host work of a batch step is spread over a
 * number of host threads (instance i on thread i mod threads; default
 * min(n, 8)); each thread steps one instance at a time.  A persistent PCG
 * launch needs all its workgroups resident at once: with T > 1 threads, a
 * launch whose grid is at most 1/(T + 1) of the workgroups the device holds
 * overlaps the launches of the other threads, a larger one waits for them
 * and they for it, so the overlapping grids always fit together.  Instances
 * are independent: a batch step gives every instance the result of
 * sisdc_step on its own with the same solver form, up to the PCG tolerance.
 *
 * sisdc_batch_handle gives the handle of instance i for the per-instance
 * calls (sisdc_set_state, sisdc_get_state, sisdc_level_info, ...); the batch
 * owns it (do not destroy it).  sisdc_batch_step steps every instance by
 * its dt[i] and fills st[i] (st may be NULL); on failure the message names
 * the first failing instance, and the other instances have still been
 * stepped.  sisdc_batch_tune is the batch's autotuner: from the current
 * states (which it restores) it times one step of every instance with each
 * solver form (persistent PCG where it fits, or multi-kernel PCG; for an
 * instance whose method asks for mixed precision also plain FP64 PCG, which
 * meets the same FP64 residual tolerance) and keeps the fastest, then times
 * whole batch steps with 1, 2, 4, 8 and 16 host threads and keeps the
 * fastest, then whole batch steps with and without step graphs
 * (sisdc_set_graph) and keeps the faster; threads_out, variants_out[n]
 * (SISDC_CG_*), precisions_out[n] (SISDC_FP64 / SISDC_MIXED) and graph_out
 * (0 / 1) receive the choices (any may be NULL).  It
 * needs a state on every instance and allocates one fine-level state copy
 * per instance while it runs. */
typedef struct sisdc_batch sisdc_batch;
int sisdc_batch_create(int n, const sisdc_problem* probs, const sisdc_method* meths, sisdc_batch** out);
int sisdc_batch_destroy(sisdc_batch* b);
int sisdc_batch_size(const sisdc_batch* b, int* n);
int sisdc_batch_handle(sisdc_batch* b, int i, sisdc_handle** h);
int sisdc_batch_set_threads(sisdc_batch* b, int threads);
int sisdc_batch_step(sisdc_batch* b, const double* dt, sisdc_stats* st);
int sisdc_batch_tune(sisdc_batch* b, const double* dt, int* threads_out, int* variants_out,
                     int* precisions_out, int* graph_out);
/* sisdc_set_graph on every instance of the batch. */
int sisdc_batch_set_graph(sisdc_batch* b, int on);

#ifdef __cplusplus
}
#endif
#endif /* SISDC_H */
