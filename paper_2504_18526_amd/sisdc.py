"""ctypes binding of libsisdc (include/sisdc.h): argument marshalling only.

Every numerical step runs in the HIP library.  Arrays may be torch tensors
on the GPU (passed as device pointers) or numpy arrays (host pointers); the
binding picks SISDC_MEM_DEVICE / SISDC_MEM_HOST accordingly.  If the shared
library has not been built the import of this module raises: there is no
fallback path.
"""
import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsisdc.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
EQ_CONVDIFF, EQ_BURGERS, EQ_EULER, EQ_NS = 0, 1, 2, 3
SI2, SI1, IMEX_EULER = 0, 1, 2
PROJ_INTERP, PROJ_L2 = 0, 1
INCREMENTAL, NONINCREMENTAL = 0, 1
NODES_RADAU_RIGHT, NODES_LOBATTO = 0, 1
START_CASCADE, START_FMG, START_PREDICTOR, START_CONSTANT = 0, 1, 2, 3
FP64, MIXED = 0, 1
CG_AUTO, CG_MULTI_KERNEL, CG_PERSISTENT_COOPERATIVE = 0, 1, 2
OP_MASS, OP_CONV, OP_FRHS, OP_SIPG, OP_HELM, OP_PROJECT, OP_INTERP, OP_RESTRICT, OP_QUAD, OP_PRECOND = range(10)
PRECOND_JACOBI, PRECOND_FDS = 0, 1

EXPORTS = [
    "sisdc_last_error", "sisdc_create", "sisdc_destroy", "sisdc_level_info",
    "sisdc_node_coords", "sisdc_set_state", "sisdc_get_level", "sisdc_set_level",
    "sisdc_get_fas", "sisdc_set_fas", "sisdc_get_state", "sisdc_update_step_params",
    "sisdc_step", "sisdc_predict", "sisdc_sweep", "mlsdc_vcycle", "helmholtz_solve", "helmholtz_solve_noalloc",
    "sisdc_apply", "sisdc_collocation_residual", "sisdc_profile_kernel",
    "sisdc_pcg_timing", "sisdc_pcg_timing_get", "sisdc_cg_kernel_timing_get", "sisdc_set_graph", "sisdc_graph_info",
    "sisdc_av_update", "sisdc_av_get",
    "sisdc_batch_create", "sisdc_batch_destroy", "sisdc_batch_size", "sisdc_batch_handle",
    "sisdc_batch_set_threads", "sisdc_batch_step", "sisdc_batch_tune", "sisdc_batch_set_graph",
    "sisdc_net_init", "sisdc_net_get_params", "sisdc_net_set_params", "sisdc_net_forward",
    "sisdc_net_train_step", "sisdc_net_grad", "sisdc_net_harvest", "sisdc_net_train", "sisdc_net_use",
]
K_SIPG_APPLY, K_SIPG_TRACE, K_CONV, K_CG_UPDATE = 0, 1, 2, 3


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_elem", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("eq", ctypes.c_int), ("a", ctypes.c_double * 3),
                ("nu", ctypes.c_double), ("gamma", ctypes.c_double),
                ("mu", ctypes.c_double), ("Pr", ctypes.c_double), ("R", ctypes.c_double),
                ("stack", ctypes.c_int)]


class Method(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("P", ctypes.c_int * 3), ("M", ctypes.c_int * 3),
                ("integrator", ctypes.c_int), ("start", ctypes.c_int),
                ("n_coarse_sweeps", ctypes.c_int), ("post_sweep", ctypes.c_int),
                ("n_iter", ctypes.c_int), ("cg_rtol", ctypes.c_double),
                ("cg_maxit", ctypes.c_int), ("c_tau", ctypes.c_double),
                ("precision", ctypes.c_int), ("cg_variant", ctypes.c_int),
                ("inner_rtol", ctypes.c_double), ("projection", ctypes.c_int), ("formulation", ctypes.c_int),
                ("nodes", ctypes.c_int), ("h_coarsen", ctypes.c_int * 3), ("c_fmg", ctypes.c_int),
                ("conserve", ctypes.c_int), ("precond", ctypes.c_int),
                ("av_kappa", ctypes.c_double), ("av_c", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("fine_sweeps", ctypes.c_int), ("solves", ctypes.c_int),
                ("cg_iters", ctypes.c_longlong), ("cg_iters_max", ctypes.c_int),
                ("not_converged", ctypes.c_int), ("max_rel_residual", ctypes.c_double),
                ("ir_rounds", ctypes.c_int), ("net_guesses", ctypes.c_int), ("net_rejected", ctypes.c_int),
                ("ir_fallbacks", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double)]


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsisdc.so is not built: run __graft_entry__.build() or "
                          "python -m paper_2504_18526_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "sisdc_last_error": ([], ctypes.c_char_p),
        "sisdc_create": ([ctypes.POINTER(Problem), ctypes.POINTER(Method), P, ctypes.POINTER(P)], I),
        "sisdc_destroy": ([P], I),
        "sisdc_level_info": ([P, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)], I),
        "sisdc_node_coords": ([P, I, P, I], I),
        "sisdc_set_state": ([P, P, I], I),
        "sisdc_get_state": ([P, P, I], I),
        "sisdc_get_level": ([P, I, P, I], I),
        "sisdc_set_level": ([P, I, P, I], I),
        "sisdc_get_fas": ([P, I, P, I], I),
        "sisdc_set_fas": ([P, I, P, I], I),
        "sisdc_update_step_params": ([P, ctypes.POINTER(D)], I),
        "sisdc_step": ([P, D, D, ctypes.POINTER(Stats)], I),
        "sisdc_predict": ([P, I, D, ctypes.POINTER(Stats)], I),
        "sisdc_sweep": ([P, I, D, P, I, ctypes.POINTER(Stats)], I),
        "mlsdc_vcycle": ([P, I, D, ctypes.POINTER(Stats)], I),
        "helmholtz_solve": ([P, I, D, P, P, P, I, D, I, ctypes.POINTER(SolveStats)], I),
        "helmholtz_solve_noalloc": ([P, I, D, P, P, P, D, I, ctypes.POINTER(SolveStats)], I),
        "sisdc_apply": ([P, I, I, D, P, P, P, I], I),
        "sisdc_collocation_residual": ([P, I, D, P, I], I),
        "sisdc_profile_kernel": ([P, I, I, D, I, ctypes.POINTER(D)], I),
        "sisdc_pcg_timing": ([P, I], I),
        "sisdc_batch_create": ([I, P, P, ctypes.POINTER(P)], I),
        "sisdc_batch_destroy": ([P], I),
        "sisdc_batch_size": ([P, ctypes.POINTER(I)], I),
        "sisdc_batch_handle": ([P, I, ctypes.POINTER(P)], I),
        "sisdc_batch_set_threads": ([P, I], I),
        "sisdc_batch_step": ([P, P, P], I),
        "sisdc_batch_tune": ([P, P, ctypes.POINTER(I), P, P, ctypes.POINTER(I)], I),
        "sisdc_batch_set_graph": ([P, I], I),
        "sisdc_set_graph": ([P, I], I),
        "sisdc_av_update": ([P], I),
        "sisdc_av_get": ([P, P, I], I),
        "sisdc_graph_info": ([P, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_longlong),
                              ctypes.POINTER(ctypes.c_longlong)], I),
        "sisdc_cg_kernel_timing_get": ([P, I, I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(D)], I),
        "sisdc_pcg_timing_get": ([P, I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                  ctypes.POINTER(D)], I),
        "sisdc_net_init": ([P, I, I, ctypes.c_ulonglong, I, I], I),
        "sisdc_net_get_params": ([P, I, P, I, ctypes.POINTER(ctypes.c_longlong)], I),
        "sisdc_net_set_params": ([P, I, P, I], I),
        "sisdc_net_forward": ([P, I, P, I, P, I, I], I),
        "sisdc_net_train_step": ([P, I, P, P, I, D, ctypes.POINTER(D), I], I),
        "sisdc_net_grad": ([P, I, P, P, I, P, ctypes.POINTER(D), I], I),
        "sisdc_net_harvest": ([P, I, I, ctypes.POINTER(I)], I),
        "sisdc_net_train": ([P, I, I, I, D, ctypes.POINTER(D)], I),
        "sisdc_net_use": ([P, I, I], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class SisdcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsisdc error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise SisdcError(rc, lib().sisdc_last_error().decode())


def _ptr(a, writable=False, dtype="float64"):
    """(pointer, mem) of a torch tensor or numpy array (contiguous, of dtype)."""
    if a is None:
        return None, MEM_DEVICE
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if str(a.dtype) != "torch." + dtype:
            raise ValueError("tensor must be " + dtype)
        if a.is_cuda:
            # the library reads and writes device buffers on its own stream:
            # work queued on the caller's current stream must finish first
            import torch
            torch.cuda.current_stream(a.device).synchronize()
        return ctypes.c_void_p(a.data_ptr()), (MEM_DEVICE if a.is_cuda else MEM_HOST)
    if not isinstance(a, np.ndarray) or a.dtype != np.dtype(dtype) or not a.flags.c_contiguous:
        raise ValueError("numpy array must be C-contiguous " + dtype)
    if writable and not a.flags.writeable:
        raise ValueError("output array is read-only")
    return ctypes.c_void_p(a.ctypes.data), MEM_HOST


def _mem_of(*arrays):
    mems = {(_ptr(a)[1]) for a in arrays if a is not None}
    if len(mems) > 1:
        raise ValueError("mixing host and device arrays in one call")
    return mems.pop() if mems else MEM_HOST


def make_problem(dim, n_elem, lo, hi, eq, a=(0.0, 0.0, 0.0), nu=0.0, gamma=1.4, mu=0.0, Pr=0.71, R=1.0, stack=1):
    """stack = B > 1: an ensemble of B instances of this problem stacked along
    the last axis (one handle, every kernel once for all instances)."""
    p = Problem()
    p.stack = stack
    p.dim = dim
    for d in range(3):
        p.n_elem[d] = n_elem[d] if d < dim else 1
        p.lo[d] = lo[d] if d < dim else 0.0
        p.hi[d] = hi[d] if d < dim else 1.0
        p.a[d] = a[d] if d < len(a) else 0.0
    p.eq = eq
    p.nu = nu
    p.gamma = gamma
    p.mu = mu
    p.Pr = Pr
    p.R = R
    return p


def make_method(P, M, integrator=SI2, start=START_CASCADE, n_coarse_sweeps=2, post_sweep=1,
                n_iter=1, cg_rtol=1e-13, cg_maxit=2000, c_tau=2.0, precision=FP64, cg_variant=CG_AUTO,
                inner_rtol=0.0, projection=PROJ_INTERP, formulation=INCREMENTAL, nodes=NODES_RADAU_RIGHT,
                h_coarsen=None, c_fmg=1, conserve=1, precond=PRECOND_JACOBI, av=None):
    m = Method()
    m.n_levels = len(P)
    for i in range(3):
        m.P[i] = P[i] if i < len(P) else 0
        m.M[i] = M[i] if i < len(M) else 0
    m.integrator = integrator
    m.start = start
    m.n_coarse_sweeps = n_coarse_sweeps
    m.post_sweep = post_sweep
    m.n_iter = n_iter
    m.cg_rtol = cg_rtol
    m.cg_maxit = cg_maxit
    m.c_tau = c_tau
    m.precision = precision
    m.cg_variant = cg_variant
    m.inner_rtol = inner_rtol
    m.projection = projection
    m.formulation = formulation
    m.nodes = nodes
    for i, v in enumerate(h_coarsen or []):
        m.h_coarsen[i] = int(v)
    m.c_fmg = c_fmg
    m.conserve = conserve
    m.precond = precond
    if av is not None:  # (kappa_s, c_s) of the artificial viscosity
        m.av_kappa, m.av_c = float(av[0]), float(av[1])
    return m


# Handles still open when the interpreter exits are closed by an exit handler,
# while the HIP runtime (and torch's use of it) is still fully alive; finalizers
# that run during interpreter teardown make no library call.
_LIVE = weakref.WeakSet()


def _close_all():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


atexit.register(_close_all)


class Solver:
    """One libsisdc handle.  Level 0 is the finest level."""

    def __init__(self, problem, method, stream=None):
        self._lib = lib()
        h = ctypes.c_void_p()
        s = ctypes.c_void_p(stream) if stream is not None else None
        _check(self._lib.sisdc_create(ctypes.byref(problem), ctypes.byref(method), s, ctypes.byref(h)))
        self.h = h
        self.problem = problem
        self.method = method
        self.dim = problem.dim
        _LIVE.add(self)

    def close(self):
        if self.h:
            self._lib.sisdc_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level=0):
        E, Np, nv, M = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.sisdc_level_info(self.h, level, ctypes.byref(E), ctypes.byref(Np),
                                          ctypes.byref(nv), ctypes.byref(M)))
        return E.value, Np.value, nv.value, M.value

    def coords(self, level=0):
        E, Np, nv, M = self.level_info(level)
        x = np.empty((self.dim, E, Np))
        _check(self._lib.sisdc_node_coords(self.h, level, x.ctypes.data_as(ctypes.c_void_p), MEM_HOST))
        return x

    def set_state(self, u0):
        p, mem = _ptr(u0)
        _check(self._lib.sisdc_set_state(self.h, p, mem))

    def get_state(self, out):
        p, mem = _ptr(out, True)
        _check(self._lib.sisdc_get_state(self.h, p, mem))
        return out

    def get_level(self, level, out):
        p, mem = _ptr(out, True)
        _check(self._lib.sisdc_get_level(self.h, level, p, mem))
        return out

    def set_level(self, level, u):
        p, mem = _ptr(u)
        _check(self._lib.sisdc_set_level(self.h, level, p, mem))

    def get_fas(self, level, out):
        p, mem = _ptr(out, True)
        _check(self._lib.sisdc_get_fas(self.h, level, p, mem))
        return out

    def set_fas(self, level, g):
        p, mem = _ptr(g)
        _check(self._lib.sisdc_set_fas(self.h, level, p, mem))

    def update_step_params(self):
        lam = ctypes.c_double()
        _check(self._lib.sisdc_update_step_params(self.h, ctypes.byref(lam)))
        return lam.value

    def step(self, dt, t=0.0):
        st = Stats()
        _check(self._lib.sisdc_step(self.h, t, dt, ctypes.byref(st)))
        return st.as_dict()

    def predict(self, level, dt):
        st = Stats()
        _check(self._lib.sisdc_predict(self.h, level, dt, ctypes.byref(st)))
        return st.as_dict()

    def sweep(self, level, dt, g=None):
        st = Stats()
        p, mem = _ptr(g) if g is not None else (None, MEM_DEVICE)
        _check(self._lib.sisdc_sweep(self.h, level, dt, p, mem, ctypes.byref(st)))
        return st.as_dict()

    def vcycle(self, top_level, dt):
        st = Stats()
        _check(self._lib.mlsdc_vcycle(self.h, top_level, dt, ctypes.byref(st)))
        return st.as_dict()

    def helmholtz_solve(self, level, dt_m, b, x, coef_state=None, rtol=0.0, maxit=0):
        mem = _mem_of(b, x, coef_state)
        st = SolveStats()
        pb, _ = _ptr(b)
        px, _ = _ptr(x, True)
        pc, _ = _ptr(coef_state)
        rc = self._lib.helmholtz_solve(self.h, level, dt_m, pc, pb, px, mem, rtol, maxit, ctypes.byref(st))
        _check(rc)
        return {"iters": st.iters, "converged": st.converged, "rel_residual": st.rel_residual}

    def helmholtz_solve_noalloc(self, level, dt_m, b, x, coef_state=None, rtol=0.0, maxit=0):
        """helmholtz_solve with the library's fixed per-GPU scratch (device
        tensors only; no allocation)."""
        if _mem_of(b, x, coef_state) != MEM_DEVICE:
            raise ValueError("helmholtz_solve_noalloc takes device arrays only")
        st = SolveStats()
        pb, _ = _ptr(b)
        px, _ = _ptr(x, True)
        pc, _ = _ptr(coef_state)
        _check(self._lib.helmholtz_solve_noalloc(self.h, level, dt_m, pc, pb, px, rtol, maxit, ctypes.byref(st)))
        return {"iters": st.iters, "converged": st.converged, "rel_residual": st.rel_residual}

    def apply(self, op, level, x, out, dt_m=0.0, aux=None):
        mem = _mem_of(x, out, aux)
        px, _ = _ptr(x)
        po, _ = _ptr(out, True)
        pa, _ = _ptr(aux)
        _check(self._lib.sisdc_apply(self.h, op, level, dt_m, px, pa, po, mem))
        return out

    def profile_kernel(self, kernel, level, dt_m, reps=200):
        us = ctypes.c_double()
        _check(self._lib.sisdc_profile_kernel(self.h, kernel, level, dt_m, reps, ctypes.byref(us)))
        return us.value

    def pcg_timing(self, on, stride=1):
        """Start (clearing the sums) or stop event timing of the persistent PCG
        launches and, in every stride-th multi-kernel solve, of the
        multi-kernel PCG's launches."""
        _check(self._lib.sisdc_pcg_timing(self.h, max(1, int(stride)) if on else 0))

    def av_update(self):
        """Evaluate the artificial viscosity from the current state."""
        _check(self._lib.sisdc_av_update(self.h))

    def av_get(self, out):
        """eps per fine element into `out` (E_fine float64 values)."""
        p, mem = _ptr(out, True)
        _check(self._lib.sisdc_av_get(self.h, p, mem))
        return out

    def set_graph(self, on):
        """Capture the step into a HIP graph and replay it (where the step
        allows it; otherwise steps run uncaptured)."""
        _check(self._lib.sisdc_set_graph(self.h, 1 if on else 0))

    def graph_info(self):
        """(last step ran through the graph, captures, graph launches)."""
        last, cap, rep = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_longlong()
        _check(self._lib.sisdc_graph_info(self.h, ctypes.byref(last), ctypes.byref(cap), ctypes.byref(rep)))
        return bool(last.value), cap.value, rep.value

    def pcg_timing_get(self, level):
        """(launches, CG iterations, total event time in us) of the persistent
        PCG launches on a level since timing was switched on."""
        n, it, us = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_double()
        _check(self._lib.sisdc_pcg_timing_get(self.h, level, ctypes.byref(n), ctypes.byref(it), ctypes.byref(us)))
        return n.value, it.value, us.value

    def cg_kernel_timing_get(self, level, kernel):
        """(launches, total event time in us) of the full-work launches of the
        multi-kernel PCG's vector update (K_CG_UPDATE) or matvec
        (K_SIPG_APPLY) on a level since timing was switched on."""
        n, us = ctypes.c_longlong(), ctypes.c_double()
        _check(self._lib.sisdc_cg_kernel_timing_get(self.h, level, kernel, ctypes.byref(n), ctypes.byref(us)))
        return n.value, us.value

    # ---- learned initial guess (element-local MLP) ----
    def net_init(self, level, hidden, seed=0, max_batch=4096, max_rows=65536):
        _check(self._lib.sisdc_net_init(self.h, level, hidden, seed, max_batch, max_rows))

    def net_params(self, level):
        n = ctypes.c_longlong()
        _check(self._lib.sisdc_net_get_params(self.h, level, None, MEM_HOST, ctypes.byref(n)))
        out = np.empty(n.value, dtype=np.float32)
        _check(self._lib.sisdc_net_get_params(self.h, level, out.ctypes.data_as(ctypes.c_void_p), MEM_HOST,
                                              ctypes.byref(n)))
        return out

    def net_set_params(self, level, theta):
        p, mem = _ptr(theta, dtype="float32")
        _check(self._lib.sisdc_net_set_params(self.h, level, p, mem))

    def net_forward(self, level, X, Y, bf16=False):
        px, mem = _ptr(X, dtype="float32")
        py, _ = _ptr(Y, True, dtype="float32")
        _check(self._lib.sisdc_net_forward(self.h, level, px, X.shape[0], py, mem, 1 if bf16 else 0))
        return Y

    def net_train_step(self, level, X, T, lr):
        px, mem = _ptr(X, dtype="float32")
        pt, _ = _ptr(T, dtype="float32")
        loss = ctypes.c_double()
        _check(self._lib.sisdc_net_train_step(self.h, level, px, pt, X.shape[0], lr, ctypes.byref(loss), mem))
        return loss.value

    def net_grad(self, level, X, T, G):
        px, mem = _ptr(X, dtype="float32")
        pt, _ = _ptr(T, dtype="float32")
        pg, _ = _ptr(G, True, dtype="float32")
        loss = ctypes.c_double()
        _check(self._lib.sisdc_net_grad(self.h, level, px, pt, X.shape[0], pg, ctypes.byref(loss), mem))
        return loss.value

    def net_harvest(self, level, on):
        rows = ctypes.c_int()
        _check(self._lib.sisdc_net_harvest(self.h, level, int(on), ctypes.byref(rows)))
        return rows.value

    def net_train(self, level, epochs, batch, lr):
        loss = ctypes.c_double()
        _check(self._lib.sisdc_net_train(self.h, level, epochs, batch, lr, ctypes.byref(loss)))
        return loss.value

    def net_use(self, level, on):
        _check(self._lib.sisdc_net_use(self.h, level, 1 if on else 0))

    def collocation_residual(self, level, dt, out):
        p, mem = _ptr(out, True)
        _check(self._lib.sisdc_collocation_residual(self.h, level, dt, p, mem))
        return out


class _Member(Solver):
    """A batch instance's handle (owned by the batch: never destroyed here)."""

    def __init__(self, batch, h, problem, method):
        self._lib = lib()
        self.h = h
        self._batch = batch  # keeps the batch alive
        self.problem = problem
        self.method = method
        self.dim = problem.dim

    def close(self):
        self.h = None


class Batch:
    """Independent instances stepped together (sisdc_batch_*)."""

    def __init__(self, problems, methods):
        self._lib = lib()
        n = len(problems)
        if n != len(methods) or n < 1:
            raise ValueError("one method per problem, at least one instance")
        self._probs = (Problem * n)(*problems)
        self._meths = (Method * n)(*methods)
        b = ctypes.c_void_p()
        _check(self._lib.sisdc_batch_create(n, ctypes.cast(self._probs, ctypes.c_void_p),
                                            ctypes.cast(self._meths, ctypes.c_void_p), ctypes.byref(b)))
        self.b = b
        self.n = n
        self.members = []
        for i in range(n):
            h = ctypes.c_void_p()
            _check(self._lib.sisdc_batch_handle(self.b, i, ctypes.byref(h)))
            self.members.append(_Member(self, h, problems[i], methods[i]))
        _LIVE.add(self)

    def close(self):
        if self.b:
            for m in self.members:
                m.h = None
            self._lib.sisdc_batch_destroy(self.b)
            self.b = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return self.n

    def __getitem__(self, i):
        return self.members[i]

    def set_threads(self, threads):
        _check(self._lib.sisdc_batch_set_threads(self.b, threads))

    def step(self, dts):
        dt = (ctypes.c_double * self.n)(*[float(d) for d in dts])
        st = (Stats * self.n)()
        _check(self._lib.sisdc_batch_step(self.b, ctypes.cast(dt, ctypes.c_void_p), ctypes.cast(st, ctypes.c_void_p)))
        return [s.as_dict() for s in st]

    def set_graph(self, on):
        _check(self._lib.sisdc_batch_set_graph(self.b, 1 if on else 0))

    def tune(self, dts, full=False):
        """Autotune the solver form of every instance, the host thread count
        and step graphs; returns (threads, [variant per instance]), or with
        `full` (threads, [variant], [precision per instance], graph)."""
        dt = (ctypes.c_double * self.n)(*[float(d) for d in dts])
        th = ctypes.c_int()
        var = (ctypes.c_int * self.n)()
        prec = (ctypes.c_int * self.n)()
        gr = ctypes.c_int()
        _check(self._lib.sisdc_batch_tune(self.b, ctypes.cast(dt, ctypes.c_void_p), ctypes.byref(th),
                                          ctypes.cast(var, ctypes.c_void_p), ctypes.cast(prec, ctypes.c_void_p),
                                          ctypes.byref(gr)))
        if full:
            return th.value, list(var), list(prec), bool(gr.value)
        return th.value, list(var)
