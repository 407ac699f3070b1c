"""Persson-Peraire artificial viscosity (test infrastructure of the CPU oracle).

The paper supplements the diffusion matrix of its DG-SEM with the artificial
viscosity of Persson and Peraire to capture shocks (Sec. 6, "Spatial
discretization"), with two parameters kappa_s and c_s per test (Sec. 8:
Burgers moving front, Sod shock tube), and refers to its references for the
details.  The form written out here is the published one (Persson & Peraire
2006: a modal smoothness sensor and a smooth switch):

    S_e   = ||u - Pi_{P-1} u||^2_e / ||u||^2_e
    s_e   = log10 S_e,         s_0 = -4 log10 P
    eps_e = 0                                        s_e < s_0 - kappa_s
          = eps_0 / 2 (1 + sin(pi (s_e - s_0) / (2 kappa_s)))   |s_e - s_0| <= kappa_s
          = eps_0                                    s_e > s_0 + kappa_s
    eps_0 = c_s (h / P) lambda_e

Readings (the paper states neither):
* u is the scalar unknown, or the density of a system;
* Pi_{P-1} is the L2 projection onto tensor polynomials of degree <= P-1 in
  every direction; both norms come from the coefficients in the orthonormal
  Legendre basis of the element (Parseval), so u - Pi_{P-1} u holds the
  modes with some index equal to P;
* h = min_d h_d, lambda_e = the largest wave speed max_d |f_c'(u)_d| over
  the element's nodes;
* eps is evaluated once per time step from u_0 on the finest level, element
  by element, and every level uses the same eps_e on its own nodes;
* eps_e enters as the diffusive flux eps_e grad u of every component: in
  F(u) as -K_{eps I} u and in the implicit coefficient D_m as + eps_e I.
"""
import numpy as np

from .element import gll_nodes_weights, legendre


def orthonormal_legendre(P, x):
    """V[i, k] = sqrt((2k + 1) / 2) P_k(x_i), k = 0..P."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([np.sqrt((2 * k + 1) / 2.0) * legendre(k, x) for k in range(P + 1)], axis=1)


def modal_coefficients(P, dim, ue):
    """Coefficients of one element's nodal values (node order x fastest) in
    the orthonormal Legendre tensor basis: solve V u_hat = u along each axis."""
    xg, _ = gll_nodes_weights(P)
    V = orthonormal_legendre(P, xg)
    n1 = P + 1
    a = np.asarray(ue, dtype=np.float64).reshape((n1,) * dim)  # axes (.., y, x)
    for ax in range(dim):
        a = np.moveaxis(np.tensordot(np.linalg.inv(V), np.moveaxis(a, ax, 0), axes=(1, 0)), 0, ax)
    return a


def smoothness(P, dim, ue):
    """S_e: share of the element's L2 energy in the modes of degree P."""
    c = modal_coefficients(P, dim, ue)
    total = float(np.sum(c * c))
    if total == 0.0:
        return 0.0
    top = np.zeros(c.shape, dtype=bool)
    for ax in range(dim):
        idx = [slice(None)] * dim
        idx[ax] = P
        top[tuple(idx)] = True
    return float(np.sum(c[top] ** 2)) / total


def switch(s, s0, kappa_s):
    """The smooth switch of eps / eps_0 as a function of s = log10 S."""
    if s < s0 - kappa_s:
        return 0.0
    if s > s0 + kappa_s:
        return 1.0
    return 0.5 * (1.0 + np.sin(np.pi * (s - s0) / (2.0 * kappa_s)))


def element_eps(mesh, phys, U, kappa_s, c_s):
    """eps_e for every element (flat element order) from the nodal state U."""
    P, dim = mesh.P, mesh.dim
    flat = mesh.to_flat(U)
    speed = np.zeros_like(U[0])
    for d in range(dim):
        speed = np.maximum(speed, phys.speed(U, d))
    speed = speed.reshape(mesh.E, mesh.Np)
    h = float(np.min(mesh.h))
    s0 = -4.0 * np.log10(P)
    eps = np.zeros(mesh.E)
    for e in range(mesh.E):
        S = smoothness(P, dim, flat[0, e])
        if S <= 0.0:
            continue
        eps[e] = c_s * (h / P) * float(np.max(speed[e])) * switch(np.log10(S), s0, kappa_s)
    return eps


def nodal(mesh, eps):
    """eps_e at every node of the element (spatial node shape of the mesh)."""
    flat = np.repeat(np.asarray(eps, dtype=np.float64)[:, None], mesh.Np, axis=1)
    return flat.reshape(mesh.shape(1)[1:])
