"""Exact solutions of the continuous problems, used as pins.

* convection-diffusion (eq. conv-diff, d dimensions, constant a, nu): each
  Fourier mode exp(2 pi i k.x) is transported with velocity a and damped by
  exp(-4 pi^2 nu |k|^2 t).
"""
import numpy as np

from paper_2504_18526_amd.inputs import fourier_modes


def convdiff_exact(coords, t, a, nu, seed=0, kmax=4):
    dim = len(coords)
    xs = [coords[d] - a[d] * t for d in range(dim)]
    u = (np.exp(-8 * np.pi ** 2 * nu * t)
         * np.sin(2 * np.pi * xs[0]) * np.sin(2 * np.pi * xs[1]))
    for k, al, be in fourier_modes(seed, dim, kmax, "normal"):
        n2 = float(sum(v * v for v in k))
        th = 2 * np.pi * sum(k[d] * xs[d] for d in range(dim))
        u = u + np.exp(-4 * np.pi ** 2 * nu * n2 * t) * (al * np.cos(th) + be * np.sin(th)) / n2
    return u
