"""SI-SDC and SI-MLSDC in the weak (dual) form, following the paper's steps.

Notation (Sec. 3 and 4): level l = 1 (coarsest) .. L (finest); on a level the
collocation nodes are t_m = t + tau_m dt, m = 1..M, with substeps
dt_m = (tau_m - tau_{m-1}) dt and u_0 the step's initial value.  A level is
any object with

    mass(x), conv(u), frhs(u), coef(u_b, dt_m, params), K(coef, x),
    solve(coef, dt_m, b, x0), tt (a temporal.TimeTable)

so the same code runs the DG discretisation and the scalar test equation.

Low-order term (eq. H_SI(1)), weak form:
    H(a, b, c) = dt_m [ C(a) - K_{D_m(b)} c ],
with D_m(b) the implicit coefficient (physics.py).  Semi-implicit systems are
solved as (M + dt_m K_{D_m(b)}) x = rhs.  The IMEX Euler term (eq. H_IMEX,
scheme "eu") is the same expression with D_m(b) = A_d(b), the physical
diffusion alone; its predictor and corrector are the one-stage forms (eqs.
sdc:incremental_predictor_eu and DeltaH_EU), i.e. those of SI(1) with that
coefficient.

Predictor SI(2) (eq. sdc:incremental_predictor_si2):
    M y   = M u_{m-1} + H(u_{m-1}, u_{m-1}, y)
    M u_m = M u_{m-1} + H(y,       u_{m-1}, u_m)
SI(1) (eq. sdc:incremental_predictor_si1) is the first line with y -> u_m.

Corrector SI(2), sweep k (eqs. sdc:incremental_corrector, DeltaH_SI2 and the
stage u^(1); with the FAS term g_m of eq. ml-sdc:incremental):
    q_m   = sum_i S_{m,i} f(u^{k-1}_i),   S = dt w^nn
    M y   = M u^k_{m-1} + q_m + g_m + H(u^k_{m-1}, u^k_{m-1}, y)
                                    - H(u^{k-1}_{m-1}, u^{k-1}_{m-1}, u^{k-1}_m)
    M u^k_m = M u^k_{m-1} + q_m + g_m + H(y, u^k_{m-1}, u^k_m)
                                    - H(u^{k-1}_m, u^{k-1}_{m-1}, u^{k-1}_m)
g_m enters both stages (reading: the paper writes the FAS term once; only
then is the collocation solution a fixed point of the two-stage sweep).
SI(1) is the first line with y -> u^k_m (eq. DeltaH_SI1).

Residual and FAS (eqs. cm:incremental:op, ml-cm:incremental:fas-mg:rhs,
MLSDC:incremental:residual):
    F_m(u) = M (u_m - u_{m-1}) - q_m(u),   r_l = g_l - F_l(u_l),
    g_{l-1} = F_{l-1}(P u_l) + R r_l,  g_L = 0.
Transfers (Sec. 4 "MLSDC transfer operators", Sec. 6 "MLSDC transfer
operators"): space-time products of 1-D Lagrange interpolation matrices,
I = I_t (x) I_x, P = P_t (x) P_x (embedded interpolation), R = I^T.
V-cycle: Alg. 2; cascade start: Alg. 3; FMG start: Alg. 4 with C_fmg V-cycles
per added level; the constant start spreads u_0 to every node of every level
and the predictor start runs the SI predictor on every level (Sec. 4,
"Multilevel algorithm").
"""
import numpy as np

from .element import RefElement, lagrange_matrix
from .temporal import TimeTable, time_transfer
from .mesh import Mesh
from .dg import DG
from . import solve as _solve
from . import av as _av


# --------------------------------------------------------------------------
# levels
# --------------------------------------------------------------------------
class DGLevel:
    """One space-time level: DG-SEM of degree P on a mesh, M Radau-right (or
    Lobatto) nodes."""

    def __init__(self, phys, n_elem, lo, hi, P, M, c_tau=2.0, rtol=1e-14,
                 maxit=20000, solver="cg", nodes="radau"):
        self.phys = phys
        self.ref = RefElement(P)
        self.mesh = Mesh(n_elem, lo, hi, P)
        self.dg = DG(self.ref, self.mesh, phys, c_tau)
        self.tt = TimeTable(M, nodes)
        self.rtol = rtol
        self.maxit = maxit
        self.solver = solver
        self.nv = phys.nv
        self.solve_log = []
        self.av = None   # artificial viscosity eps_e at the nodes (av.py), set per step

    def shape(self):
        return self.mesh.shape(self.nv)

    def mass(self, x):
        return self.dg.mass(x)

    def conv(self, u):
        return self.dg.conv(u)

    def frhs(self, u):
        if self.av is None:
            return self.dg.frhs(u)
        # with artificial viscosity the diffusive flux is (nu + eps_e) grad u
        # (scalar equations) or eps_e grad u of every component (systems)
        out = self.dg.conv(u)
        nu = 0.0 if self.phys.system else self.phys.nu
        out = out - self.dg.sipg(self._iso(nu + self.av), u)
        if getattr(self.phys, "mu", 0.0) != 0.0:
            out = out + self.dg.visc(u)
        return out

    def _iso(self, field):
        dim = self.mesh.dim
        Dc = np.zeros((dim, dim) + np.shape(field))
        for d in range(dim):
            Dc[d, d] = field
        return Dc

    def _with_av(self, Dc):
        if self.av is None:
            return Dc
        Dc = Dc.copy()
        for d in range(self.mesh.dim):
            Dc[d, d] = Dc[d, d] + self.av
        return Dc

    def coef(self, ub, dtm, params):
        return self._with_av(self.phys.coef(ub, dtm, params))

    def coef_d(self, ub, dtm, params):
        return self._with_av(self.phys.coef_d(ub, dtm, params))

    def K(self, Dc, x):
        return self.dg.sipg(Dc, x)

    def solve(self, Dc, dtm, b, x0):
        apply = lambda x: self.dg.helmholtz(Dc, dtm, x)
        if self.solver == "dense":
            x = _solve.dense_solve(apply, b)
            self.solve_log.append((0, 0.0))
            return x
        pre = self.dg.Wm * np.ones_like(b)
        x, it, rel = _solve.cg(apply, b, x0, pre, rtol=self.rtol, maxit=self.maxit)
        self.solve_log.append((it, rel))
        return x

    def coords(self):
        return self.mesh.node_coords(self.ref.x)


class SpaceTransfer:
    """p-coarsening transfer between two DG levels on the same mesh:
    I_x (coarse -> fine), P_x (fine -> coarse) and R_x = I_x^T, each a 1-D
    matrix applied along every axis.  P_x (Sec. 4, "MLSDC transfer
    operators", eq. projection_int and the choice that follows it) is either
    embedded interpolation (the coarse nodal values of the fine polynomial)
    or the L^2 projection onto the coarse polynomials of each element:
    P = (I^T W_f I)^-1 I^T W_f per axis, with W_f the fine GLL weights (the
    fine quadrature integrates the coarse mass matrix exactly for P_c < P_f;
    the element Jacobian cancels)."""

    def __init__(self, fine, coarse, projection="interp"):
        self.fine, self.coarse = fine, coarse
        self.I1 = lagrange_matrix(coarse.ref.x, fine.ref.x)     # (Pf+1, Pc+1)
        if projection == "interp":
            self.P1 = lagrange_matrix(fine.ref.x, coarse.ref.x)     # (Pc+1, Pf+1)
        elif projection == "l2":
            Wf = np.diag(fine.ref.w)
            self.P1 = np.linalg.solve(self.I1.T @ Wf @ self.I1, self.I1.T @ Wf)
        else:
            raise ValueError(projection)

    def _apply(self, X, A):
        mesh = self.fine.mesh
        for d in range(mesh.dim):
            ax = mesh.node_axis(d)
            X = np.moveaxis(np.tensordot(A, X, axes=([1], [ax])), 0, ax)
        return X

    def I(self, xc):
        return self._apply(xc, self.I1)

    def P(self, xf):
        return self._apply(xf, self.P1)

    def R(self, rf):
        return self._apply(rf, self.I1.T)


class SpaceTransferH:
    """2:1 h-coarsening in space (Sec. 6, "MLSDC transfer operators"), with
    p-coarsening on top: every coarse element fuses 2 fine elements along
    each axis.  Each operator is a 1-D matrix on an axis' "pair" of fine
    elements (2 (Pf+1) nodes, left child first) applied along every axis:

    * I (coarse -> fine): each child evaluates the coarse polynomial at its
      nodes, xi_c = (xi_f - 1)/2 (left child) or (xi_f + 1)/2 (right);
    * R = I^T (each coarse element sums its children's contributions);
    * P (fine -> coarse), embedded interpolation: each coarse node takes the
      value of the child containing it.  Before that the jump between the
      two children is removed by linear blending (reading of the paper's
      default adjustment): with J the right child's value at the shared
      face minus the left child's, the left child gets + J/2 (xi_c + 1) and
      the right child - J/2 (1 - xi_c), so both meet at the mean there (the
      paper's averaged centre contribution) and the outer faces keep their
      values;
    * P, L^2 projection: both children contribute to the whole coarse
      element, P = (I^T W I)^-1 I^T W with W = diag(w_f / 2, w_f / 2)."""

    def __init__(self, fine, coarse, projection="interp"):
        self.fine, self.coarse = fine, coarse
        xf, xc = np.asarray(fine.ref.x), np.asarray(coarse.ref.x)
        nf, nc = len(xf), len(xc)
        self.I1 = np.vstack([lagrange_matrix(xc, (xf - 1.0) / 2.0),
                             lagrange_matrix(xc, (xf + 1.0) / 2.0)])       # (2 nf, nc)
        if projection == "interp":
            B = np.zeros((nc, 2 * nf))
            for j, x in enumerate(xc):
                if x < 0.0:
                    B[j, :nf] = lagrange_matrix(xf, np.array([2.0 * x + 1.0]))[0]
                    phi = 0.5 * (x + 1.0)                 # blending weight J/2 * (x + 1)
                elif x > 0.0:
                    B[j, nf:] = lagrange_matrix(xf, np.array([2.0 * x - 1.0]))[0]
                    phi = -0.5 * (1.0 - x)
                else:                                     # the shared centre: the mean of both children
                    B[j, nf - 1] += 0.5
                    B[j, nf] += 0.5
                    continue
                # + phi * J, J = u_right(first node) - u_left(last node)
                B[j, nf] += phi
                B[j, nf - 1] -= phi
            self.P1 = B
        elif projection == "l2":
            W = np.diag(np.concatenate([fine.ref.w, fine.ref.w]) / 2.0)
            self.P1 = np.linalg.solve(self.I1.T @ W @ self.I1, self.I1.T @ W)
        else:
            raise ValueError(projection)

    def _f2c(self, X, A):
        """A (nc x 2 nf) along every axis: fine-level array -> coarse."""
        mesh = self.fine.mesh
        for d in range(mesh.dim):
            ea, na = mesh.elem_axis(d), mesh.node_axis(d)
            X = np.moveaxis(X, (ea, na), (-2, -1))
            sh = X.shape
            X = X.reshape(sh[:-2] + (sh[-2] // 2, 2 * sh[-1])) @ A.T
            X = np.moveaxis(X, (-2, -1), (ea, na))
        return X

    def _c2f(self, X, A):
        """A (2 nf x nc) along every axis: coarse-level array -> fine."""
        mesh = self.fine.mesh
        for d in range(mesh.dim):
            ea, na = mesh.elem_axis(d), mesh.node_axis(d)
            X = np.moveaxis(X, (ea, na), (-2, -1))
            Y = X @ A.T                                   # (..., nc_elem, 2 nf)
            sh = Y.shape
            X = Y.reshape(sh[:-2] + (sh[-2] * 2, sh[-1] // 2))
            X = np.moveaxis(X, (-2, -1), (ea, na))
        return X

    def I(self, xc):
        return self._c2f(xc, self.I1)

    def P(self, xf):
        return self._f2c(xf, self.P1)

    def R(self, rf):
        return self._f2c(rf, self.I1.T)


# --------------------------------------------------------------------------
# single-level building blocks
# --------------------------------------------------------------------------
def substeps(lv, dt):
    return dt * lv.tt.dtau


def quadrature(lv, F, dt):
    """q_m = sum_i S_{m,i} f_i, S = dt w^nn (eq. cm:incremental).  F holds
    f at nodes 1..M; returns q for nodes 1..M (index 0 unused: None)."""
    S = lv.tt.S(dt)
    M = lv.tt.M
    q = [None]
    for m in range(M):
        acc = np.zeros_like(F[1])
        for i in range(M):
            acc = acc + S[m, i] * F[i + 1]
        q.append(acc)
    return q


def implicit_coef(lv, ub, dtm, params, scheme):
    """D_m(u_b) of the low-order term: (dt_m/2) A_c^2 + A_d (SI, eq. H_SI(1))
    or A_d alone (IMEX Euler, eq. H_IMEX)."""
    if scheme == "eu":
        return lv.coef_d(ub, dtm, params)
    return lv.coef(ub, dtm, params)


def one_stage(scheme):
    return scheme in ("si1", "eu")


def H(lv, a, b, c, dtm, params, scheme="si2"):
    """Weak H(a, b, c) = dt_m [C(a) - K_{D_m(b)} c]."""
    return dtm * (lv.conv(a) - lv.K(implicit_coef(lv, b, dtm, params, scheme), c))


def predictor(lv, u0, dt, params, scheme="si2"):
    """SI(1) / SI(2) / IMEX Euler predictor sweep: returns [u_0, u_1, ..., u_M]."""
    U = [u0]
    dts = substeps(lv, dt)
    for m in range(1, lv.tt.M + 1):
        dtm = dts[m - 1]
        ua = U[m - 1]
        Dc = implicit_coef(lv, ua, dtm, params, scheme)
        y = lv.solve(Dc, dtm, lv.mass(ua) + dtm * lv.conv(ua), ua)
        if one_stage(scheme):
            U.append(y)
            continue
        U.append(lv.solve(Dc, dtm, lv.mass(ua) + dtm * lv.conv(y), y))
    return U


def sweep(lv, U, dt, params, g=None, scheme="si2"):
    """One incremental SI(1)/SI(2)/IMEX Euler corrector sweep (Alg. 1 with N = 1)."""
    M = lv.tt.M
    dts = substeps(lv, dt)
    F = [None] + [lv.frhs(U[i]) for i in range(1, M + 1)]
    q = quadrature(lv, F, dt)
    Unew = [U[0]]
    for m in range(1, M + 1):
        dtm = dts[m - 1]
        h1_old = H(lv, U[m - 1], U[m - 1], U[m], dtm, params, scheme)
        ua = Unew[m - 1]
        Dc = implicit_coef(lv, ua, dtm, params, scheme)
        base = lv.mass(ua) + q[m]
        if g is not None:
            base = base + g[m]
        y = lv.solve(Dc, dtm, base + dtm * lv.conv(ua) - h1_old, U[m])
        if one_stage(scheme):
            Unew.append(y)
            continue
        h2_old = H(lv, U[m], U[m - 1], U[m], dtm, params, scheme)
        Unew.append(lv.solve(Dc, dtm, base + dtm * lv.conv(y) - h2_old, y))
    return Unew


def collocation_residual(lv, U, dt):
    """F_m(u) = M (u_m - u_{m-1}) - q_m(u), m = 1..M (index 0: None)."""
    M = lv.tt.M
    F = [None] + [lv.frhs(U[i]) for i in range(1, M + 1)]
    q = quadrature(lv, F, dt)
    return [None] + [lv.mass(U[m] - U[m - 1]) - q[m] for m in range(1, M + 1)]


# --------------------------------------------------------------------------
# non-incremental (zero-to-node) form (Sec. 3 "Non-incremental SDC method",
# Sec. 4 "Non-incremental multilevel SDC method")
# --------------------------------------------------------------------------
def quadrature0n(lv, F, dt):
    """q0n_m = dt sum_i w0n_{m,i} f_i (eq. cm:non-incremental)."""
    W = dt * lv.tt.w0n
    M = lv.tt.M
    q = [None]
    for m in range(M):
        acc = 0.0
        for i in range(M):
            acc = acc + W[m, i] * F[i + 1]
        q.append(acc)
    return q


def sweep0n(lv, U, dt, params, g0n=None, scheme="si2"):
    """One zero-to-node sweep (eq. sdc:non-incremental; with the FAS term of
    eq. ml-sdc:non-incremental:matrix):
        M u^k_m = M u_0 + q0n_m + g0n_m + sum_{i<=m} DeltaH^k_i,
    the deltas the same as in the incremental form.  The SI(2) stage keeps
    its incremental definition (the paper states it only in that form), with
    the node's share g0n_m - g0n_{m-1} of the FAS term (reading)."""
    M = lv.tt.M
    dts = substeps(lv, dt)
    F = [None] + [lv.frhs(U[i]) for i in range(1, M + 1)]
    q0 = quadrature0n(lv, F, dt)
    qn = quadrature(lv, F, dt)
    Unew = [U[0]]
    acc = 0.0                                     # sum of the deltas of nodes 1..m-1
    base0 = lv.mass(U[0])
    for m in range(1, M + 1):
        dtm = dts[m - 1]
        ua = Unew[m - 1]
        Dc = implicit_coef(lv, ua, dtm, params, scheme)
        g_m = g0n[m] if g0n is not None else 0.0
        g_prev = g0n[m - 1] if (g0n is not None and m > 1) else 0.0
        h1_old = H(lv, U[m - 1], U[m - 1], U[m], dtm, params, scheme)
        rhs0 = base0 + q0[m] + g_m + acc
        if one_stage(scheme):
            # DeltaH_m = H(ua, ua, u_m) - h1_old, implicit in u_m
            um = lv.solve(Dc, dtm, rhs0 + dtm * lv.conv(ua) - h1_old, U[m])
            acc = acc + H(lv, ua, ua, um, dtm, params, scheme) - h1_old
            Unew.append(um)
            continue
        stage = lv.mass(ua) + qn[m] + (g_m - g_prev)
        y = lv.solve(Dc, dtm, stage + dtm * lv.conv(ua) - h1_old, U[m])
        h2_old = H(lv, U[m], U[m - 1], U[m], dtm, params, scheme)
        um = lv.solve(Dc, dtm, rhs0 + dtm * lv.conv(y) - h2_old, y)
        acc = acc + H(lv, y, ua, um, dtm, params, scheme) - h2_old
        Unew.append(um)
    return Unew


def collocation_residual0n(lv, U, dt):
    """F0n_m(u) = M (u_m - u_0) - q0n_m(u), m = 1..M (eq. cm:non-incremental:matrix)."""
    M = lv.tt.M
    F = [None] + [lv.frhs(U[i]) for i in range(1, M + 1)]
    q = quadrature0n(lv, F, dt)
    return [None] + [lv.mass(U[m] - U[0]) - q[m] for m in range(1, M + 1)]


# --------------------------------------------------------------------------
# space-time transfers
# --------------------------------------------------------------------------
class Transfer:
    """Space-time transfer between level l (fine) and l-1 (coarse)."""

    def __init__(self, fine, coarse, space=None, projection="interp"):
        self.fine, self.coarse = fine, coarse
        self.It, self.Pt, self.Rt = time_transfer(fine.tt, coarse.tt)
        if space is None:
            same = tuple(fine.mesh.n) == tuple(coarse.mesh.n)
            space = SpaceTransfer(fine, coarse, projection) if same else SpaceTransferH(fine, coarse, projection)
        self.space = space

    def interp(self, Uc):
        """(I_t (x) I_x) on nodes 1..M_c -> nodes 1..M_f (index 0: None)."""
        Mf, Mc = self.fine.tt.M, self.coarse.tt.M
        xs = [None] + [self.space.I(Uc[j]) for j in range(1, Mc + 1)]
        out = [None]
        for i in range(Mf):
            acc = 0.0
            for j in range(Mc):
                acc = acc + self.It[i, j] * xs[j + 1]
            out.append(acc)
        return out

    def project(self, Uf):
        Mf, Mc = self.fine.tt.M, self.coarse.tt.M
        xs = [None] + [self.space.P(Uf[j]) for j in range(1, Mf + 1)]
        out = [None]
        for i in range(Mc):
            acc = 0.0
            for j in range(Mf):
                acc = acc + self.Pt[i, j] * xs[j + 1]
            out.append(acc)
        return out

    def restrict(self, rf):
        Mf, Mc = self.fine.tt.M, self.coarse.tt.M
        xs = [None] + [self.space.R(rf[i]) for i in range(1, Mf + 1)]
        out = [None]
        for j in range(Mc):
            acc = 0.0
            for i in range(Mf):
                acc = acc + self.It[i, j] * xs[i + 1]
            out.append(acc)
        return out


# --------------------------------------------------------------------------
# multilevel driver
# --------------------------------------------------------------------------
class MLSDC:
    """SI-MLSDC on levels[0] (l = 1, coarsest) .. levels[L-1] (l = L)."""

    def __init__(self, levels, transfers=None, scheme="si2", n_coarse=2,
                 start="cascade", cycles=3, post_sweep=True, c_fmg=1, projection="interp",
                 formulation="incremental", av=None):
        self.levels = levels
        self.av = av  # (kappa_s, c_s) of the artificial viscosity (av.py), or None
        if formulation not in ("incremental", "nonincremental"):
            raise ValueError(formulation)
        self.nonincremental = formulation == "nonincremental"
        self.L = len(levels)
        if transfers is None:
            transfers = [None] + [Transfer(levels[i], levels[i - 1], projection=projection)
                                  for i in range(1, self.L)]
        self.tr = transfers            # tr[i]: between levels[i] and levels[i-1]
        self.scheme = scheme
        self.n_coarse = n_coarse
        self.start = start
        self.cycles = cycles
        self.post_sweep = post_sweep
        self.c_fmg = c_fmg
        self.U = [None] * self.L
        self.g = [None] * self.L
        self.v = [None] * self.L
        self.u0 = [None] * self.L
        self.params = None

    # ---- pieces --------------------------------------------------------
    def set_initial(self, u0_fine, params):
        """u_{l,0}: the fine initial value, projected level by level
        (reading: the coarse initial values are P_x of the fine one)."""
        self.params = params
        self.u0[self.L - 1] = u0_fine
        for i in range(self.L - 1, 0, -1):
            self.u0[i - 1] = self.tr[i].space.P(self.u0[i])

    def sdc_sweep(self, i, dt, g):
        sw = sweep0n if self.nonincremental else sweep
        self.U[i] = sw(self.levels[i], self.U[i], dt, self.params, g, self.scheme)

    def residual_op(self, lv, U, dt):
        return (collocation_residual0n if self.nonincremental else collocation_residual)(lv, U, dt)

    def vcycle(self, top, dt):
        """Alg. 2 on levels[0..top]; the top level has g = 0."""
        self.g[top] = None
        for i in range(top, 0, -1):
            lv, lc, tr = self.levels[i], self.levels[i - 1], self.tr[i]
            self.sdc_sweep(i, dt, self.g[i])                          # pre-sweep
            Fl = self.residual_op(lv, self.U[i], dt)
            r = [None] + [(self.g[i][m] if self.g[i] is not None else 0.0) - Fl[m]
                          for m in range(1, lv.tt.M + 1)]             # residual
            v = tr.project(self.U[i])                                 # restriction
            v[0] = self.u0[i - 1]
            self.v[i - 1] = v
            Fc = self.residual_op(lc, v, dt)
            Rr = tr.restrict(r)
            self.g[i - 1] = [None] + [Fc[m] + Rr[m] for m in range(1, lc.tt.M + 1)]
            self.U[i - 1] = list(v)
        for _ in range(self.n_coarse):                                # coarse solve
            self.sdc_sweep(0, dt, self.g[0])
        for i in range(1, top + 1):
            tr = self.tr[i]
            diff = [None] + [self.U[i - 1][m] - self.v[i - 1][m]
                             for m in range(1, self.levels[i - 1].tt.M + 1)]
            corr = tr.interp(diff)                                    # prolongation
            self.U[i] = [self.U[i][0]] + [self.U[i][m] + corr[m]
                                          for m in range(1, self.levels[i].tt.M + 1)]
            if i < top:
                self.sdc_sweep(i, dt, self.g[i])                      # post-sweep

    def interpolate_up(self, i):
        """u_{l+1} <- I u_l on nodes 1..M (the initial value stays)."""
        up = self.tr[i + 1].interp(self.U[i])
        self.U[i + 1] = [self.u0[i + 1]] + up[1:]

    def start_levels(self, dt):
        L = self.L
        if self.start == "predictor":
            for i in range(L):
                self.U[i] = predictor(self.levels[i], self.u0[i], dt, self.params, self.scheme)
            return
        if self.start == "constant":                                  # u_0 spread to every node
            for i in range(L):
                self.U[i] = [self.u0[i]] * (self.levels[i].tt.M + 1)
            return
        self.U[0] = predictor(self.levels[0], self.u0[0], dt, self.params, self.scheme)
        if L == 1:
            return
        if self.start == "cascade":                                   # Alg. 3
            for i in range(0, L - 1):
                self.sdc_sweep(i, dt, None)
                self.interpolate_up(i)
        elif self.start == "fmg":                                     # Alg. 4
            self.sdc_sweep(0, dt, None)
            self.interpolate_up(0)
            for i in range(1, L - 1):
                for _ in range(self.c_fmg):
                    self.vcycle(i, dt)
                self.interpolate_up(i)
        else:
            raise ValueError(self.start)

    def step(self, u0_fine, dt):
        """One time step; returns u at t + dt (u_{L,M}, Radau right)."""
        params = self.levels[-1].phys.step_params(u0_fine) \
            if hasattr(self.levels[-1], "phys") else None
        if self.av is not None:  # eps_e from u_0 on the finest level, used on every level
            fine = self.levels[-1]
            eps = _av.element_eps(fine.mesh, fine.phys, u0_fine, *self.av)
            for lv in self.levels:
                if lv.mesh.n != fine.mesh.n:
                    raise ValueError("artificial viscosity needs the same elements on every level")
                lv.av = _av.nodal(lv.mesh, eps)
        self.set_initial(u0_fine, params)
        self.start_levels(dt)
        if self.L == 1:
            for _ in range(self.cycles):
                self.sdc_sweep(0, dt, None)
        else:
            for _ in range(self.cycles):
                self.vcycle(self.L - 1, dt)
            if self.post_sweep:
                self.sdc_sweep(self.L - 1, dt, None)
        return self.U[self.L - 1][-1]


def sdc_step(lv, u0, dt, sweeps, scheme="si2"):
    """Single-level SI-SDC step: predictor and `sweeps` corrector sweeps."""
    params = lv.phys.step_params(u0) if hasattr(lv, "phys") else None
    U = predictor(lv, u0, dt, params, scheme)
    for _ in range(sweeps):
        U = sweep(lv, U, dt, params, None, scheme)
    return U[-1]
