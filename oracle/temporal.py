"""Collocation in time (Sec. 3, "Single-level collocation and SDC methods";
Sec. 4, "MLSDC transfer operators").

* nodes   : t_m = t + tau_m dt, m = 1..M, tau_M = 1.  Radau right (the
            default): the left end point t_0 is not a collocation node; tau
            are the roots of P_M(x) - P_{M-1}(x) mapped from [-1, 1] to
            [0, 1].  Lobatto: both end points are nodes (tau_1 = 0, so
            u_1 = u_0); tau are the M Gauss-Lobatto points.
* w^nn    : incremental (node-to-node) weights, eq. (nn_weights):
            w^nn_{m,i} = (1/dt) int_{t_{m-1}}^{t_m} l_i(t) dt, with l_i the
            Lagrange basis on t_1..t_M and t_0 = t.
* S       : S = dt * w^nn  (the "S-matrix" of the node quadrature).
* w^0n    : zero-to-node weights, eq. (0n_weights): cumulative row sums.
* I_t     : coarse-to-fine interpolation, I_t[i, j] = l^c_j(tau^f_i).
* P_t     : fine-to-coarse embedded interpolation, P_t[i, j] = l^f_j(tau^c_i).
* R_t     : residual restriction, the transpose of I_t (eq. restriction).
"""
import numpy as np
from numpy.polynomial import legendre as npleg

from .element import lagrange_matrix


def radau_right_nodes(M):
    """Radau IIA nodes on [0, 1] (ascending, last node = 1)."""
    if M < 1:
        raise ValueError("M >= 1 required")
    if M == 1:
        return np.array([1.0])
    c = np.zeros(M + 1)
    c[M] = 1.0
    c[M - 1] -= 1.0
    r = np.sort(np.real(npleg.legroots(c)))
    # Newton polish on P_M - P_{M-1}
    dc = npleg.legder(c)
    for _ in range(5):
        r = r - npleg.legval(r, c) / npleg.legval(r, dc)
    r[-1] = 1.0
    return (r + 1.0) / 2.0


def lobatto_nodes(M):
    """Lobatto IIIA nodes on [0, 1]: the M Gauss-Lobatto-Legendre points."""
    if M < 2:
        raise ValueError("M >= 2 required for Lobatto nodes")
    from .element import gll_nodes_weights
    x, _ = gll_nodes_weights(M - 1)
    t = (np.asarray(x) + 1.0) / 2.0
    t[0], t[-1] = 0.0, 1.0
    return t


def _gauss_legendre(n):
    x, w = npleg.leggauss(n)
    return x, w


def nn_weights(tau):
    """w^nn[m, i] = int_{tau_{m-1}}^{tau_m} l_i(s) ds on [0, 1] (tau_0 = 0).

    Integrated with an (M+1)-point Gauss-Legendre rule, exact for the
    degree M-1 Lagrange polynomials.
    """
    M = len(tau)
    xg, wg = _gauss_legendre(M + 1)
    W = np.zeros((M, M))
    lo = 0.0
    for m in range(M):
        hi = tau[m]
        s = lo + (hi - lo) * (xg + 1.0) / 2.0
        L = lagrange_matrix(tau, s)          # L[q, i] = l_i(s_q)
        W[m, :] = (hi - lo) / 2.0 * (wg @ L)
        lo = hi
    return W


def zero_to_node_weights(Wnn):
    """w^0n[m, i] = sum_{j <= m} w^nn[j, i] (eq. 0n_weights)."""
    return np.cumsum(Wnn, axis=0)


class TimeTable:
    """Collocation tables for M Radau-right (or Lobatto) nodes on the unit
    interval."""

    def __init__(self, M, nodes="radau"):
        self.M = int(M)
        if nodes == "radau":
            self.tau = radau_right_nodes(self.M)
        elif nodes == "lobatto":
            self.tau = lobatto_nodes(self.M)
        else:
            raise ValueError(nodes)
        self.wnn = nn_weights(self.tau)
        self.w0n = zero_to_node_weights(self.wnn)
        # substep lengths (fractions of dt): dtau_m = tau_m - tau_{m-1}
        self.dtau = np.diff(np.concatenate(([0.0], self.tau)))

    def S(self, dt):
        """S = dt * w^nn."""
        return dt * self.wnn


def time_transfer(tt_fine, tt_coarse):
    """(I_t, P_t, R_t) between two node sets of the same kind (Sec. 4)."""
    I_t = lagrange_matrix(tt_coarse.tau, tt_fine.tau)    # M_f x M_c
    P_t = lagrange_matrix(tt_fine.tau, tt_coarse.tau)    # M_c x M_f
    return I_t, P_t, I_t.T.copy()
