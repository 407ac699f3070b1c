"""Seeded synthetic inputs: initial fields evaluated at given coordinates.

This module holds no arithmetic of the numerical method.  Every function
takes physical node coordinates (computed by the caller from its own
reference element) and returns field values, so the same seeded data feed
both the HIP library and the CPU checker.

Recipes (periodic boxes, analytic data shaped like the paper's test
problems, which are all analytic; no dataset is involved):

* fourier_modes   : wave vectors k in Z^d over a half space (first non-zero
                    component positive) with 0 < |k| <= kmax, coefficients
                    drawn from numpy.random.default_rng(seed).
* convdiff_field  : sin(2 pi x) sin(2 pi y) + sum_k (a_k cos 2pi k.x
                    + b_k sin 2pi k.x) / |k|^2, a_k, b_k ~ N(0, 1).
* burgers_field   : sum_k cos(2 pi k.x + phi_k) / |k|^2, phi_k ~ U[0, 2pi),
                    scaled so that max |u| over the given points is 1.
* isentropic_vortex : Euler state of a vortex of strength eps on a uniform
                    background rho = p = 1 moving along +x at Mach `mach`.
* taylor_green    : 3-D Taylor-Green state for the Navier-Stokes case.
"""
import numpy as np


def fourier_modes(seed, dim, kmax, kind="normal"):
    rng = np.random.default_rng(seed)
    ks = []
    rng_k = range(-kmax, kmax + 1)
    grids = np.array(np.meshgrid(*([list(rng_k)] * dim), indexing="ij")).reshape(dim, -1).T
    for k in grids:
        k = tuple(int(v) for v in k)
        n2 = sum(v * v for v in k)
        if n2 == 0 or n2 > kmax * kmax:
            continue
        first = next(v for v in k if v != 0)
        if first < 0:
            continue
        ks.append(k)
    ks.sort(key=lambda k: (sum(v * v for v in k), k))
    modes = []
    for k in ks:
        if kind == "normal":
            modes.append((k, float(rng.standard_normal()), float(rng.standard_normal())))
        else:
            modes.append((k, float(rng.uniform(0.0, 2.0 * np.pi)), 0.0))
    return modes


def _phase(coords, k):
    return 2.0 * np.pi * sum(k[d] * coords[d] for d in range(len(k)))


def convdiff_field(coords, seed=0, kmax=4):
    """Initial field of the convection-diffusion case at the given points."""
    dim = len(coords)
    u = np.sin(2 * np.pi * coords[0]) * np.sin(2 * np.pi * coords[1])
    for k, a, b in fourier_modes(seed, dim, kmax, "normal"):
        n2 = float(sum(v * v for v in k))
        th = _phase(coords, k)
        u = u + (a * np.cos(th) + b * np.sin(th)) / n2
    return u


def convdiff_exact(coords, t, a, nu, seed=0, kmax=4):
    """The convection-diffusion field of convdiff_field after time t of
    u_t + a.grad u = nu lap u on the periodic unit box: every Fourier mode k
    moves with a and decays by exp(-nu (2 pi |k|)^2 t)."""
    dim = len(coords)
    xs = [coords[d] - a[d] * t for d in range(dim)]
    decay = lambda n2: np.exp(-nu * 4.0 * np.pi * np.pi * n2 * t)
    u = np.sin(2 * np.pi * xs[0]) * np.sin(2 * np.pi * xs[1]) * decay(2.0)
    for k, ak, bk in fourier_modes(seed, dim, kmax, "normal"):
        n2 = float(sum(v * v for v in k))
        th = _phase(xs, k)
        u = u + (ak * np.cos(th) + bk * np.sin(th)) / n2 * decay(n2)
    return u


def burgers_field(coords, seed=0, kmax=6):
    """Initial field of the Burgers case, max |u| = 1 over the points."""
    dim = len(coords)
    u = np.zeros_like(coords[0])
    for k, phi, _ in fourier_modes(seed, dim, kmax, "phase"):
        n2 = float(sum(v * v for v in k))
        u = u + np.cos(_phase(coords, k) + phi) / n2
    return u / np.max(np.abs(u))


def isentropic_vortex(coords, t=0.0, eps=5.0, mach=0.5, gamma=1.4,
                      centre=(5.0, 5.0), length=(10.0, 10.0)):
    """Conservative Euler state (rho, rho u, rho v, rho e) of the isentropic
    vortex translated with the background flow to time t (periodic box;
    the nearest periodic image of the centre is used)."""
    x, y = coords[0], coords[1]
    uinf = mach * np.sqrt(gamma)
    xc = centre[0] + uinf * t
    dx = x - xc
    dy = y - centre[1]
    dx = dx - length[0] * np.round(dx / length[0])
    dy = dy - length[1] * np.round(dy / length[1])
    r2 = dx * dx + dy * dy
    du = eps / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * (-dy)
    dv = eps / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * dx
    T = 1.0 - (gamma - 1.0) * eps * eps / (8 * gamma * np.pi * np.pi) * np.exp(1 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    u = uinf + du
    v = dv
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


def taylor_green(coords, mach=0.1, gamma=1.4, rho0=1.0, V0=1.0):
    """Conservative Navier-Stokes state (rho, rho u, rho v, rho w, rho e) of
    the Taylor-Green vortex on [0, 2 pi]^3 with uniform temperature."""
    x, y, z = coords
    p0 = rho0 * V0 * V0 / (gamma * mach * mach)
    u = V0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -V0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(x)
    p = p0 + rho0 * V0 * V0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    T0 = p0 / rho0                     # R = 1
    rho = p / T0
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def sod_pair(coords, h, gamma=1.4, width=0.2):
    """Periodic pair of Sod shock tubes on [0, 2] (x only): the left state of
    Sod's problem (rho = 1, p = 1, v = 0) on [0, 1), the right state (rho =
    0.125, p = 0.1) on [1, 2), each jump smoothed by a tanh of width `width`
    h (h the element size).  Until the two wave systems meet, [0.5, 1.5]
    holds Sod's tube with its diaphragm at x = 1.  Returns the conserved
    state (4, ...)."""
    import numpy as np
    x = np.asarray(coords[0], dtype=np.float64)
    w = 0.5 * (np.tanh(x / (width * h)) - np.tanh((x - 1.0) / (width * h))
               + np.tanh((x - 2.0) / (width * h)) + 1.0)
    w = np.clip(w, 0.0, 1.0)
    rho = 0.125 + 0.875 * w
    p = 0.1 + 0.9 * w
    zero = np.zeros_like(rho)
    return np.stack([rho, zero, zero, p / (gamma - 1.0)])
