"""Shared set-up for the parity tests: the same discretisation built once as
an oracle level (CPU, FP64) and once as a libsisdc handle (GPU)."""
import numpy as np

from oracle import sdc as osdc
from oracle.physics import ConvDiff, Burgers, Euler, NavierStokes


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


NS_MU, NS_PR = 0.02, 0.71


def oracle_phys(eq, dim, a=(1.0, 0.5, 0.25), nu=0.01, gamma=1.4):
    if eq == "convdiff":
        return ConvDiff(list(a[:dim]), nu)
    if eq == "burgers":
        return Burgers(dim, nu)
    if eq == "ns":
        return NavierStokes(dim, gamma, NS_MU, NS_PR)
    return Euler(dim, gamma)


def lib_problem(S, eq, dim, n, lo, hi, a=(1.0, 0.5, 0.25), nu=0.01, gamma=1.4):
    code = {"convdiff": S.EQ_CONVDIFF, "burgers": S.EQ_BURGERS, "euler": S.EQ_EULER, "ns": S.EQ_NS}[eq]
    return S.make_problem(dim, n, lo, hi, code, a=a[:dim], nu=nu, gamma=gamma, mu=NS_MU, Pr=NS_PR)


def random_state(phys, mesh, rng, amp=1.0):
    """Random nodal state valid for the equation (positive density and
    pressure for Euler)."""
    shp = mesh.shape(phys.nv)
    if phys.nv == 1:
        return amp * rng.standard_normal(shp)
    dim = phys.dim
    U = np.empty(shp)
    rho = 1.0 + 0.2 * rng.random(shp[1:])
    v = [0.3 * rng.standard_normal(shp[1:]) for _ in range(dim)]
    p = 1.0 + 0.2 * rng.random(shp[1:])
    U[0] = rho
    for k in range(dim):
        U[1 + k] = rho * v[k]
    U[dim + 1] = p / (phys.gamma - 1.0) + 0.5 * rho * sum(vk * vk for vk in v)
    return U


def smooth_state(phys, level, rng):
    """Smooth field for the equation on the level's nodes."""
    x = level.coords()
    dim = phys.dim
    if phys.nv == 1:
        th = 2 * np.pi * sum((d + 1) * x[d] / (level.mesh.hi[d] - level.mesh.lo[d]) for d in range(dim))
        return (0.6 * np.sin(th) + 0.3 * np.cos(2 * np.pi * x[0] / (level.mesh.hi[0] - level.mesh.lo[0])) + 0.2)[None]
    L = [level.mesh.hi[d] - level.mesh.lo[d] for d in range(dim)]
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * x[0] / L[0]) * np.cos(2 * np.pi * x[1] / L[1])
    v = [0.2 * np.cos(2 * np.pi * x[(d + 1) % dim] / L[(d + 1) % dim]) for d in range(dim)]
    p = 1.0 + 0.1 * np.cos(2 * np.pi * x[0] / L[0])
    U = np.empty((dim + 2,) + x[0].shape)
    U[0] = rho
    for k in range(dim):
        U[1 + k] = rho * v[k]
    U[dim + 1] = p / (phys.gamma - 1.0) + 0.5 * rho * sum(vk * vk for vk in v)
    return U
