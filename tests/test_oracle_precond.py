"""Pins of the oracle's element-block Jacobi preconditioner (oracle/precond.py).

* The diagonal block A_ee of M + dt_m K_{kappa I}, assembled by brute force
  from the matrix-free operator, is symmetric positive definite, and equals
  the Kronecker sum J (W x W (x W) + dt_m kappa sum_d K_d x W ...) of one-axis
  matrices written here from the interior-penalty form of Sec. 6 (volume
  term and the element's own face terms, penalty C_tau (P+1)^2 kappa / h):
  the separable structure that fast diagonalisation relies on.
* PCG with the block preconditioner reaches the dense solution, in fewer
  iterations than point Jacobi on a diffusion-dominated system.
CPU only."""
import numpy as np
import pytest

from oracle.element import RefElement
from oracle.mesh import Mesh
from oracle.dg import DG
from oracle import precond, solve


def axis_matrix(P, h, c_tau=2.0):
    """One-axis part of the element block per unit diffusivity and unit weight
    of the other axes: (2/h)^2 [D^T W D - 1/2 sum_s n_s (D^T e_s e_s^T +
    e_s e_s^T D) + 1/2 C_tau (P+1)^2 sum_s e_s e_s^T], s the end nodes with
    outward normals n = -1 (node 0) and +1 (node P)."""
    ref = RefElement(P)
    D, W = ref.D, np.diag(ref.w)
    n = P + 1
    K = D.T @ W @ D
    for e, nrm in ((0, -1.0), (P, 1.0)):
        E = np.zeros((n, n))
        E[e, e] = 1.0
        K = K - 0.5 * nrm * (D.T @ E + E @ D) + 0.5 * c_tau * n * n * E
    return (2.0 / h) ** 2 * K, W


@pytest.mark.parametrize("P,h", [(3, (0.3, 0.5)), (4, (0.25, 0.25)), (2, (0.4, 0.3, 0.7)), (3, (0.5, 0.5, 0.5))])
def test_element_block_is_the_kronecker_sum(P, h):
    kappa, dtm = 0.7, 0.05
    A = precond.element_block(P, h, kappa, dtm)
    assert np.max(np.abs(A - A.T)) < 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T))[0] > 0.0
    dim = len(h)
    J = float(np.prod(np.asarray(h) / 2.0))
    Ks, Ws = zip(*[axis_matrix(P, hd) for hd in h])
    # node index: x fastest, so the x factor is the last Kronecker factor
    def kron(mats):
        out = mats[0]
        for m in mats[1:]:
            out = np.kron(out, m)
        return out
    mass = kron([Ws[d] for d in reversed(range(dim))])
    # every term carries the element Jacobian J; K_d is per unit of J and of the other axes' weights
    stiff = sum(kron([Ks[d] if e == d else Ws[e] for e in reversed(range(dim))]) for d in range(dim))
    expect = J * (mass + dtm * kappa * stiff)
    assert np.max(np.abs(A - expect)) < 1e-11 * np.abs(expect).max()


def test_block_jacobi_pcg_reaches_the_dense_solution():
    P, n, h = 3, (3, 4), (0.25, 0.2)
    kappa, dtm = 0.5, 0.08
    ref = RefElement(P)
    mesh = Mesh(n, [0, 0], [n[0] * h[0], n[1] * h[1]], P)

    class _Phys:
        nv = 1
        system = True

    dg = DG(ref, mesh, _Phys())
    Dc = precond.iso_tensor(2, kappa, mesh.shape(1)[1:])
    apply = lambda x: dg.helmholtz(Dc, dtm, x)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(mesh.shape(1))
    x_dense = solve.dense_solve(apply, b)
    A_ee = precond.element_block(P, h, kappa, dtm)
    pre = lambda r: precond.block_jacobi(mesh, A_ee, r)
    x_b, it_b, rel_b = solve.cg(apply, b, np.zeros_like(b), pre, rtol=1e-13)
    x_j, it_j, rel_j = solve.cg(apply, b, np.zeros_like(b), dg.Wm * np.ones_like(b), rtol=1e-13)
    assert np.linalg.norm(x_b - x_dense) < 1e-11 * np.linalg.norm(x_dense)
    assert np.linalg.norm(x_j - x_dense) < 1e-11 * np.linalg.norm(x_dense)
    assert it_b < it_j, (it_b, it_j)
