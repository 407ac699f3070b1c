"""Equations: fluxes, wave speeds and implicit (diffusion) coefficients.

Problem statement (Sec. 2, "Problem"): u_t + div f_c(u) = div f_d(u, grad u)
(+ sources, none used here).  The semi-implicit low-order terms H^SI
(Sec. 3, eq. H_SI(1)) treat  div((dt_m / 2) A_c(u_b)^2 + A_d(u_b)) grad u_c
implicitly; in d > 1 dimensions the scalar Lax-Wendroff form of that
coefficient is the tensor  (dt_m / 2) a a^T + nu I  with a = f_c'(u_b)
(reading: the multi-d extension of the paper's 1-D term).

For systems (Euler / Navier-Stokes) the coefficient (dt_m/2) A_c^2 is not
symmetric, so it is replaced by a constant isotropic artificial diffusion
kappa_m I with kappa_m = (dt_m / 2) lam*^2, lam* the largest max_d(|v_d|+c)
over the nodes of the step's initial value (reading for systems; the
Navier-Stokes case adds the largest of 4 mu / (3 rho) and gamma mu / (Pr rho)).
Because H enters the corrector only as a difference of two evaluations, the
choice does not change the collocation solution the sweeps converge to.
"""
import numpy as np


class ConvDiff:
    """Linear convection-diffusion u_t + div(a u) = nu lap u (eq. conv-diff)."""
    nv = 1
    system = False

    def __init__(self, a, nu):
        self.a = np.asarray(a, dtype=np.float64)
        self.dim = len(self.a)
        self.nu = float(nu)

    def flux(self, U, d):
        return self.a[d] * U

    def speed(self, U, d):
        return np.abs(self.a[d]) * np.ones_like(U[0])

    def coef(self, Ub, dtm, params=None):
        """Tensor (dt_m/2) a a^T + nu I at every node: shape (d, d) + node shape."""
        shp = Ub[0].shape
        Dc = np.zeros((self.dim, self.dim) + shp)
        for i in range(self.dim):
            for j in range(self.dim):
                Dc[i, j] = 0.5 * dtm * self.a[i] * self.a[j] + (self.nu if i == j else 0.0)
        return Dc

    def coef_d(self, Ub, dtm, params=None):
        """A_d alone (IMEX Euler, eq. H_IMEX): nu I at every node."""
        shp = Ub[0].shape
        Dc = np.zeros((self.dim, self.dim) + shp)
        for i in range(self.dim):
            Dc[i, i] = self.nu
        return Dc

    def step_params(self, U0):
        return None


class Burgers:
    """Viscous Burgers u_t + div((u^2/2) (1,..,1)) = nu lap u (eq. burgers,
    source term zero)."""
    nv = 1
    system = False

    def __init__(self, dim, nu):
        self.dim = int(dim)
        self.nu = float(nu)

    def flux(self, U, d):
        return 0.5 * U * U

    def speed(self, U, d):
        return np.abs(U[0])

    def coef(self, Ub, dtm, params=None):
        """(dt_m/2) u_b^2 (1,..,1)(1,..,1)^T + nu I."""
        u2 = Ub[0] * Ub[0]
        Dc = np.zeros((self.dim, self.dim) + u2.shape)
        for i in range(self.dim):
            for j in range(self.dim):
                Dc[i, j] = 0.5 * dtm * u2 + (self.nu if i == j else 0.0)
        return Dc

    def coef_d(self, Ub, dtm, params=None):
        """A_d alone (IMEX Euler, eq. H_IMEX): nu I at every node."""
        shp = Ub[0].shape
        Dc = np.zeros((self.dim, self.dim) + shp)
        for i in range(self.dim):
            Dc[i, i] = self.nu
        return Dc

    def step_params(self, U0):
        return None


class Euler:
    """Compressible Euler equations in conservative variables
    (rho, rho v_1..rho v_d, rho e_t), perfect gas (Sec. 2, "Euler and
    Navier-Stokes equations", written for d dimensions)."""
    system = True

    def __init__(self, dim, gamma, R=1.0):
        self.dim = int(dim)
        self.nv = self.dim + 2
        self.gamma = float(gamma)
        self.R = float(R)

    def primitive(self, U):
        rho = U[0]
        v = [U[1 + k] / rho for k in range(self.dim)]
        ke = 0.5 * sum(vk * vk for vk in v)
        p = (self.gamma - 1.0) * (U[self.dim + 1] - rho * ke)
        return rho, v, p

    def flux(self, U, d):
        rho, v, p = self.primitive(U)
        F = np.empty_like(U)
        F[0] = U[1 + d]
        for k in range(self.dim):
            F[1 + k] = U[1 + k] * v[d] + (p if k == d else 0.0)
        F[self.dim + 1] = (U[self.dim + 1] + p) * v[d]
        return F

    def sound_speed(self, U):
        rho, v, p = self.primitive(U)
        return np.sqrt(self.gamma * p / rho)

    def speed(self, U, d):
        rho, v, p = self.primitive(U)
        return np.abs(v[d]) + np.sqrt(self.gamma * p / rho)

    def step_params(self, U0):
        """lam* = max over nodes of max_d (|v_d| + c) at the step's u_0."""
        lam = max(float(np.max(self.speed(U0, d))) for d in range(self.dim))
        return {"lam": lam, "visc": 0.0}

    def kappa(self, dtm, params):
        return 0.5 * dtm * params["lam"] ** 2 + params["visc"]

    def coef_d(self, Ub, dtm, params):
        """A_d alone (IMEX Euler, eq. H_IMEX): zero.  The Euler equations have
        no diffusion; the Navier-Stokes viscous term stays explicit inside f
        (reading), so IMEX Euler substeps of a system are explicit apart from
        the mass matrix."""
        shp = Ub[0].shape
        return np.zeros((self.dim, self.dim) + shp)

    def coef(self, Ub, dtm, params):
        kap = self.kappa(dtm, params)
        shp = Ub[0].shape
        Dc = np.zeros((self.dim, self.dim) + shp)
        for i in range(self.dim):
            Dc[i, i] = kap
        return Dc


class NavierStokes(Euler):
    """Compressible Navier-Stokes (Sec. 2, "Euler and Navier-Stokes
    equations", written for d dimensions): constant dynamic viscosity mu,
    Prandtl number Pr, perfect gas with gas constant R.

    Viscous flux in direction d:  (0, tau_1d, ..., tau_Dd,
    sum_k v_k tau_kd + lam_T dT/dx_d), with the Newtonian stress
    tau_ij = mu (dv_j/dx_i + dv_i/dx_j) - 2/3 mu delta_ij div v and the heat
    conductivity lam_T = mu c_p / Pr, c_p = gamma R / (gamma - 1).  In 1-D
    this is the paper's f_d = (0, 4/3 eta v_x, 4/3 eta v v_x + lambda T_x).

    Implicit coefficient (reading for systems): kappa_m = (dt_m/2) lam*^2 +
    max(4 mu / (3 rho_min), gamma mu / (Pr rho_min)), lam* and rho_min taken
    over the nodes of the step's initial value.
    """

    def __init__(self, dim, gamma, mu, Pr, R=1.0):
        super().__init__(dim, gamma, R)
        self.mu = float(mu)
        self.Pr = float(Pr)
        self.cp = self.gamma * self.R / (self.gamma - 1.0)
        self.lam_T = self.mu * self.cp / self.Pr

    def step_params(self, U0):
        lam = max(float(np.max(self.speed(U0, d))) for d in range(self.dim))
        rho_min = float(np.min(U0[0]))
        visc = max(4.0 * self.mu / (3.0 * rho_min), self.gamma * self.mu / (self.Pr * rho_min))
        return {"lam": lam, "visc": visc}

    def primitive_q(self, U):
        """q = (v_1, ..., v_D, T), the variables whose gradients enter f_d."""
        rho, v, p = self.primitive(U)
        return np.stack(v + [p / (rho * self.R)])

    def viscous_flux(self, U, G, d):
        """f_v,d from the state U and the gradients G[e][j] = d q_j / dx_e."""
        D = self.dim
        rho, v, p = self.primitive(U)
        div = sum(G[k][k] for k in range(D))
        tau_d = [self.mu * (G[i][d] + G[d][i]) - (2.0 / 3.0 * self.mu * div if i == d else 0.0)
                 for i in range(D)]
        F = np.zeros_like(U)
        for i in range(D):
            F[1 + i] = tau_d[i]
        F[D + 1] = sum(v[k] * tau_d[k] for k in range(D)) + self.lam_T * G[d][D]
        return F
