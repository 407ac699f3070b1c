"""Element-block Jacobi preconditioner of the implicit Helmholtz system (test
infrastructure of the CPU oracle).

The paper compares PCG with a fast-diagonalisation solver in its runtime
analysis (Sec. 8, "Runtime analysis").  Here the element-wise solve serves
as the preconditioner of the PCG: z_e = A_ee^-1 r_e for every element e,
with A_ee the diagonal block of A = M + dt_m K_D that couples the element's
nodes with themselves.  The plain definition is used: A_ee is assembled by
applying the matrix-free operator to unit vectors supported on one element
and reading that element's rows; on a uniform periodic mesh with a constant
coefficient every element has the same block.  The preconditioner changes
the PCG iterates only, never the solution.
"""
import numpy as np

from .dg import DG
from .element import RefElement
from .mesh import Mesh


def iso_tensor(dim, kappa, shape):
    """kappa I at every node (shape: the spatial shape of a nodal array)."""
    Dc = np.zeros((dim, dim) + tuple(shape))
    for d in range(dim):
        Dc[d, d] = kappa
    return Dc


def element_block(P, h, kappa, dtm, c_tau=2.0):
    """Dense A_ee (N_p x N_p, node order x fastest) of M + dtm K_{kappa I} for
    elements of size h (one entry per axis), built on a periodic mesh of 3
    elements per axis so that the element's neighbours are other elements."""
    dim = len(h)
    n = (3,) * dim
    ref = RefElement(P)
    mesh = Mesh(n, [0.0] * dim, [3.0 * hd for hd in h], P)

    class _Phys:
        nv = 1
        system = True

    dg = DG(ref, mesh, _Phys(), c_tau)
    shp = mesh.shape(1)
    Dc = iso_tensor(dim, kappa, shp[1:])
    Np = mesh.Np
    A = np.zeros((Np, Np))
    X = np.zeros(shp)
    for j in range(Np):
        flat = X.reshape(1, mesh.E, Np)
        flat[0, 0, j] = 1.0
        Y = dg.helmholtz(Dc, dtm, X)
        A[:, j] = Y.reshape(1, mesh.E, Np)[0, 0]
        flat[0, 0, j] = 0.0
    return A


def block_jacobi(level_mesh, A_ee, R):
    """z = A_ee^-1 r for every (component, element) of the nodal array R."""
    nv = R.shape[0]
    flat = R.reshape(nv * level_mesh.E, level_mesh.Np)
    Z = np.linalg.solve(A_ee, flat.T).T
    return Z.reshape(R.shape)
