"""Periodic uniform Cartesian mesh and the tensor layout of nodal arrays.

The paper's discretisation (Sec. 6) splits the domain into elements; the
configurations here are periodic boxes split into n_1 x ... x n_d equal
elements of size h_d.  The map from the reference element [-1, 1]^d is
affine, so the Jacobian J = prod_d h_d / 2 is constant.

Nodal arrays have the shape

    (n_v, n_{d-1}, ..., n_0, P+1, ..., P+1)

i.e. variable, element index (slowest axis first) and node index (slowest
axis first).  Reshaped in C order to (n_v, E, N_p) this is the flat layout
u[var][elem][node] with elem = e_0 + n_0 (e_1 + n_1 e_2) and
node = i_0 + (P+1) (i_1 + (P+1) i_2): the x direction is fastest.
"""
import numpy as np


class Mesh:
    def __init__(self, n_elem, lo, hi, P):
        self.dim = len(n_elem)
        self.n = tuple(int(v) for v in n_elem)
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.h = (self.hi - self.lo) / np.asarray(self.n, dtype=np.float64)
        self.P = int(P)
        self.J = float(np.prod(self.h / 2.0))
        self.E = int(np.prod(self.n))
        self.Np = (self.P + 1) ** self.dim

    # axis bookkeeping ---------------------------------------------------
    def elem_axis(self, d):
        """Array axis of the element index along direction d."""
        return 1 + (self.dim - 1 - d)

    def node_axis(self, d):
        """Array axis of the node index along direction d."""
        return 1 + self.dim + (self.dim - 1 - d)

    def shape(self, nv):
        return (nv,) + tuple(reversed(self.n)) + (self.P + 1,) * self.dim

    def to_flat(self, U):
        return U.reshape(U.shape[0], self.E, self.Np)

    def from_flat(self, u, nv=None):
        u = np.asarray(u)
        if nv is None:
            nv = u.shape[0]
        return u.reshape(self.shape(nv))

    # geometry -----------------------------------------------------------
    def node_coords(self, xi):
        """Physical coordinates of all nodes: a list over d of arrays of
        shape (n_{d-1}, ..., n_0, P+1, ..., P+1); xi are the reference
        nodes on [-1, 1] (affine map of each element)."""
        full = self.shape(1)[1:]
        coords = []
        for d in range(self.dim):
            e = np.arange(self.n[d], dtype=np.float64)
            x = self.lo[d] + self.h[d] * (e[:, None] + (np.asarray(xi)[None, :] + 1.0) / 2.0)
            shp = [1] * (2 * self.dim)
            shp[self.elem_axis(d) - 1] = self.n[d]
            shp[self.node_axis(d) - 1] = self.P + 1
            coords.append(np.broadcast_to(x.reshape(shp), full).copy())
        return coords

    def mass_weights(self, w):
        """Diagonal of the GLL-lumped mass matrix, J * w_i w_j (w_k),
        shaped to broadcast against a nodal array (leading var axis)."""
        Wn = np.ones((self.P + 1,) * self.dim)
        for d in range(self.dim):
            shp = [1] * self.dim
            shp[self.dim - 1 - d] = self.P + 1
            Wn = Wn * w.reshape(shp)
        return (self.J * Wn).reshape((1,) + (1,) * self.dim + (self.P + 1,) * self.dim)

    def face_weights(self, w, d):
        """J_f * prod of tangential weights for a face normal to d, shaped
        like a face slice (node axis d removed)."""
        Jf = float(np.prod([self.h[k] / 2.0 for k in range(self.dim) if k != d]))
        Wf = np.ones((self.P + 1,) * (self.dim - 1))
        others = [k for k in range(self.dim) if k != d]        # ascending dims
        # face slice node axes are the remaining node axes, slowest first
        for pos, k in enumerate(reversed(others)):
            shp = [1] * (self.dim - 1)
            shp[pos] = self.P + 1
            Wf = Wf * w.reshape(shp)
        return (Jf * Wf).reshape((1,) + (1,) * self.dim + (self.P + 1,) * (self.dim - 1))
