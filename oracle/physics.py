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

    def coef(self, Ub, dtm, params):
        kap = self.kappa(dtm, params)
        shp = Ub[0].shape
        Dc = np.zeros((self.dim, self.dim) + shp)
        for i in range(self.dim):
            Dc[i, i] = kap
        return Dc
