"""The scalar test equation form of SI-SDC / SI-MLSDC (Sec. 5, eq. dahlquist).

For a Fourier mode exp(i k x) of the convection-diffusion equation the
operators reduce to numbers: the convective part is i lam_i, the diffusion
lam_r (lam_r = -nu k^2, lam_i = -v k), and the implicit coefficient
(dt_m/2) A_c^2 + A_d acts as K = (dt_m/2) lam_i^2 - lam_r (IMEX Euler:
A_d alone, K = -lam_r).  The mass is 1.
Plugging these into the same predictor / corrector / V-cycle code gives the
stability function R(z) = u^{n+1} / u^n, z = dt (lam_r + i lam_i).
"""
import numpy as np

from .temporal import TimeTable, time_transfer
from . import sdc


class DahlquistLevel:
    def __init__(self, lam_r, lam_i, M, nodes="radau"):
        self.lam_r = float(lam_r)
        self.lam_i = float(lam_i)
        self.tt = TimeTable(M, nodes)

    def mass(self, x):
        return x

    def conv(self, u):
        return 1j * self.lam_i * u

    def frhs(self, u):
        return (self.lam_r + 1j * self.lam_i) * u

    def coef(self, ub, dtm, params):
        return 0.5 * dtm * self.lam_i ** 2 - self.lam_r

    def coef_d(self, ub, dtm, params):
        """A_d alone (IMEX Euler): the diffusion -lam_r."""
        return -self.lam_r

    def K(self, c, x):
        return c * x

    def solve(self, c, dtm, b, x0):
        return b / (1.0 + dtm * c)


class _Identity:
    def I(self, x):
        return x

    def P(self, x):
        return x

    def R(self, x):
        return x


def mlsdc(lam_r, lam_i, Ms, nodes="radau", **kw):
    levels = [DahlquistLevel(lam_r, lam_i, M, nodes) for M in Ms]
    tr = [None] + [sdc.Transfer(levels[i], levels[i - 1], space=_Identity())
                   for i in range(1, len(levels))]
    return sdc.MLSDC(levels, tr, **kw)


def amplification_sdc(z, M, sweeps, scheme="si2", nodes="radau"):
    """R(z) of single-level SDC with `sweeps` corrector sweeps, dt = 1."""
    lv = DahlquistLevel(z.real, z.imag, M, nodes)
    return complex(sdc.sdc_step(lv, np.complex128(1.0), 1.0, sweeps, scheme))


def amplification_mlsdc(z, Ms, cycles, **kw):
    ml = mlsdc(z.real, z.imag, Ms, cycles=cycles, **kw)
    return complex(ml.step(np.complex128(1.0), 1.0))
