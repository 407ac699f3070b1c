"""Nodal DG-SEM weak operators on a periodic Cartesian mesh (Sec. 6).

All operators return vectors in the weak ("dual") form: the value at node i
is the functional tested against the Lagrange basis function of node i, as in
the discrete collocation equation (eq. collocation:radau-iia:full), where
every term is a functional of the weighting function w_h.

* mass      M x: GLL-collocated quadrature, diagonal (reading: lumped mass).
* conv      C(u) = F_c(w, u): -int w div f_c(u) - sum_faces int w (f* - f(u^-)).n
            in strong DG-SEM form with a local Lax-Friedrichs numerical flux
            f*.n = 1/2 (f(u^-) + f(u^+)).n - 1/2 lam (u^+ - u^-),
            lam = max of the directional wave speed on both sides
            (reading: the paper defers the flux to its companion paper).
* sipg      K_D x: symmetric interior penalty form of -div(D grad x) with a
            node-wise symmetric tensor D,
              a(w, x) = sum_e int grad w . D grad x
                      - sum_f int {D grad x}.n [w] - sum_f int {D grad w}.n [x]
                      + sum_f int tau [x][w],
            [x] = x^- - x^+ along n = n^-, tau = C_tau (P+1)^2 kappa_f / h_d,
            kappa_f = max(n.D^- n, n.D^+ n) per face node (reading).
* visc      V(u): weak viscous term of Navier-Stokes by the first Bassi-Rebay
            scheme (reading: the paper defers F_d to its companion paper):
            lifted gradients G = grad q + M^-1 sum_faces E^T J_f W_f ({q} - q^-) n
            of q = (v, T), nodal viscous fluxes f_v(u, G), then
            V = int w div f_v + sum_faces int w ({f_v} - f_v^-).n, central
            averages on both sides.
* frhs      F(u) = C(u) - K_{nu I} u for the scalar equations, C(u) for Euler,
            C(u) + V(u) for Navier-Stokes.

Integrals use the GLL nodes of each element (collocated quadrature).
"""
import numpy as np


class DG:
    """Weak DG-SEM operators for one discretisation level."""

    def __init__(self, ref, mesh, phys, c_tau=2.0):
        self.ref = ref
        self.mesh = mesh
        self.phys = phys
        self.dim = mesh.dim
        self.nv = phys.nv
        self.P = ref.P
        self.c_tau = float(c_tau)
        self.Wm = mesh.mass_weights(ref.w)
        self.Wf = [mesh.face_weights(ref.w, d) for d in range(self.dim)]

    # --- tensor helpers --------------------------------------------------
    def deriv(self, X, d):
        """(D X) along reference direction d (no metric factor)."""
        ax = self.mesh.node_axis(d)
        return np.moveaxis(np.tensordot(self.ref.D, X, axes=([1], [ax])), 0, ax)

    def deriv_T(self, X, d):
        """(D^T X) along reference direction d."""
        ax = self.mesh.node_axis(d)
        return np.moveaxis(np.tensordot(self.ref.D.T, X, axes=([1], [ax])), 0, ax)

    def face(self, X, d, side, lead=1):
        """Face slice of X (node index 0 for side -1, P for side +1) and the
        matching slice of the neighbour across that face.

        lead = number of leading non-spatial axes of X (1 for a nodal array
        with a variable axis, 0 for a bare spatial field)."""
        ax = self.mesh.node_axis(d) - 1 + lead
        eax = self.mesh.elem_axis(d) - 1 + lead
        own_idx = 0 if side < 0 else self.P
        nb_idx = self.P if side < 0 else 0
        own = np.take(X, own_idx, axis=ax)
        nb = np.roll(np.take(X, nb_idx, axis=ax), 1 if side < 0 else -1, axis=eax)
        return own, nb

    def face_add(self, out, val, d, side):
        sl = [slice(None)] * out.ndim
        sl[self.mesh.node_axis(d)] = 0 if side < 0 else self.P
        out[tuple(sl)] += val

    # --- operators -------------------------------------------------------
    def mass(self, X):
        return self.Wm * X

    def conv(self, U):
        """C(u): weak convective operator with the LLF interface flux."""
        phys, mesh = self.phys, self.mesh
        vol = np.zeros_like(U)
        for d in range(self.dim):
            vol -= (2.0 / mesh.h[d]) * self.deriv(phys.flux(U, d), d)
        out = self.Wm * vol
        for d in range(self.dim):
            for side in (-1, 1):
                u_in, u_out = self.face(U, d, side)
                fin = side * phys.flux(u_in, d)
                fout = side * phys.flux(u_out, d)
                lam = np.maximum(phys.speed(u_in, d), phys.speed(u_out, d))
                fstar = 0.5 * (fin + fout) - 0.5 * lam[None] * (u_out - u_in)
                self.face_add(out, -self.Wf[d] * (fstar - fin), d, side)
        return out

    def sipg(self, Dc, X):
        """K_D x for each variable of X with the node-wise tensor Dc
        (shape (d, d) + spatial shape), the same for every variable."""
        mesh, dim = self.mesh, self.dim
        G = [(2.0 / mesh.h[d]) * self.deriv(X, d) for d in range(dim)]
        Qf = [sum(Dc[d, e][None] * G[e] for e in range(dim)) for d in range(dim)]  # D grad x
        Q = [self.Wm * Qf[d] for d in range(dim)]
        out = np.zeros_like(X)
        Pp1sq = (self.P + 1) ** 2
        for d in range(dim):
            for side in (-1, 1):
                x_in, x_out = self.face(X, d, side)
                q_in, q_out = self.face(Qf[d], d, side)
                k_in, k_out = self.face(Dc[d, d], d, side, lead=0)
                qn_mean = 0.5 * side * (q_in + q_out)          # {D grad x}.n
                tau = self.c_tau * Pp1sq * np.maximum(k_in, k_out) / mesh.h[d]
                jump = x_in - x_out
                self.face_add(out, self.Wf[d] * (-qn_mean + tau[None] * jump), d, side)
                # symmetry term: -1/2 [x] (D^- n) . grad w, lifted through D^T
                for e in range(dim):
                    dn_e = side * np.take(Dc[e, d], 0 if side < 0 else self.P,
                                          axis=mesh.node_axis(d) - 1)
                    self.face_add(Q[e], -0.5 * self.Wf[d] * jump * dn_e[None], d, side)
        for d in range(dim):
            out += (2.0 / mesh.h[d]) * self.deriv_T(Q[d], d)
        return out

    def nu_tensor(self):
        """nu I at every node (physical diffusion of the scalar equations)."""
        shp = self.mesh.shape(1)[1:]
        Dc = np.zeros((self.dim, self.dim) + shp)
        for d in range(self.dim):
            Dc[d, d] = self.phys.nu
        return Dc

    def lifted_gradients(self, U):
        """BR1 gradients G[e][j] = d q_j / dx_e of q = (v, T) per node."""
        phys, mesh = self.phys, self.mesh
        q = phys.primitive_q(U)
        G = [[None] * q.shape[0] for _ in range(self.dim)]
        for e in range(self.dim):
            ge = (2.0 / mesh.h[e]) * self.deriv(q, e)
            for side in (-1, 1):
                q_in, q_out = self.face(q, e, side)
                # (J_f w_f / (J w)) at the face node equals (2 / h_e) / w_face
                w_face = self.ref.w[0 if side < 0 else self.P]
                self.face_add(ge, (2.0 / mesh.h[e]) / w_face * 0.5 * (q_out - q_in) * side, e, side)
            for j in range(q.shape[0]):
                G[e][j] = ge[j]
        return G

    def visc(self, U):
        """V(u): weak BR1 viscous term (Navier-Stokes)."""
        phys, mesh = self.phys, self.mesh
        G = self.lifted_gradients(U)
        Fv = [phys.viscous_flux(U, G, d) for d in range(self.dim)]
        vol = np.zeros_like(U)
        for d in range(self.dim):
            vol += (2.0 / mesh.h[d]) * self.deriv(Fv[d], d)
        out = self.Wm * vol
        for d in range(self.dim):
            for side in (-1, 1):
                f_in, f_out = self.face(Fv[d], d, side)
                self.face_add(out, self.Wf[d] * 0.5 * side * (f_out - f_in), d, side)
        return out

    def frhs(self, U):
        """F(u) = F_c + F_d (eq. collocation:radau-iia:full), weak form."""
        out = self.conv(U)
        if not self.phys.system and self.phys.nu != 0.0:
            out = out - self.sipg(self.nu_tensor(), U)
        if getattr(self.phys, "mu", 0.0) != 0.0:
            out = out + self.visc(U)
        return out

    def helmholtz(self, Dc, dtm, X):
        """A x = M x + dt_m K_D x."""
        return self.mass(X) + dtm * self.sipg(Dc, X)

    # --- diagnostics -----------------------------------------------------
    def integral(self, U):
        """int u dx per variable (GLL quadrature): sum of M u."""
        return (self.Wm * U).reshape(U.shape[0], -1).sum(axis=1)

    def l2(self, U):
        return np.sqrt((self.Wm * U * U).reshape(U.shape[0], -1).sum(axis=1))
