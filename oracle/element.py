"""Gauss-Lobatto-Legendre (GLL) reference element on [-1, 1].

The paper's spatial discretisation (Sec. 6, "Spatial discretization") uses
polynomials of degree P in each element; the nodal basis sits on the P+1
GLL points.  These are textbook constructions, written out plainly:

* nodes  : -1, 1 and the roots of P_P'(x) (derivative of the Legendre
           polynomial of degree P)
* weights: w_j = 2 / (P (P+1) P_P(x_j)^2)
* D_ij   = l_j'(x_i) for the Lagrange basis l_j on the nodes (barycentric)
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def legendre(n, x):
    """Legendre polynomial P_n evaluated at x (three-term recurrence)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p1


def gll_nodes_weights(P):
    """GLL nodes (ascending) and quadrature weights for degree P >= 1."""
    if P < 1:
        raise ValueError("P >= 1 required")
    # interior nodes: roots of P_P'
    cP = np.zeros(P + 1)
    cP[P] = 1.0
    dcoef = npleg.legder(cP)
    interior = np.sort(np.real(npleg.legroots(dcoef))) if P > 1 else np.array([])
    x = np.concatenate(([-1.0], interior, [1.0]))
    # polish interior roots by Newton on P_P'(x) = 0
    d2coef = npleg.legder(dcoef)
    for _ in range(5):
        if P > 1:
            xi = x[1:-1]
            xi = xi - npleg.legval(xi, dcoef) / npleg.legval(xi, d2coef)
            x[1:-1] = xi
    w = 2.0 / (P * (P + 1) * legendre(P, x) ** 2)
    return x, w


def barycentric_weights(x):
    """Barycentric weights lambda_j = 1 / prod_{k != j} (x_j - x_k)."""
    n = len(x)
    lam = np.ones(n)
    for j in range(n):
        for k in range(n):
            if k != j:
                lam[j] /= (x[j] - x[k])
    return lam


def derivative_matrix(x):
    """D_ij = l_j'(x_i): derivative of the Lagrange basis on nodes x."""
    n = len(x)
    lam = barycentric_weights(x)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def lagrange_matrix(x_from, x_to):
    """L[i, j] = l_j(x_to[i]) for the Lagrange basis l_j on nodes x_from.

    Evaluates the interpolant through x_from at the points x_to.  Written as
    the plain product formula (no barycentric shortcut), exact for points
    that coincide with a node.
    """
    x_from = np.asarray(x_from, dtype=np.float64)
    x_to = np.asarray(x_to, dtype=np.float64)
    L = np.zeros((len(x_to), len(x_from)))
    for i, t in enumerate(x_to):
        for j, xj in enumerate(x_from):
            v = 1.0
            for k, xk in enumerate(x_from):
                if k != j:
                    v *= (t - xk) / (xj - xk)
            L[i, j] = v
    return L


class RefElement:
    """GLL reference element of degree P: nodes, weights, derivative."""

    def __init__(self, P):
        self.P = int(P)
        self.n = self.P + 1
        self.x, self.w = gll_nodes_weights(self.P)
        self.D = derivative_matrix(self.x)
