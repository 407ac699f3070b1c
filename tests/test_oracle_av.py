"""Pins of the oracle's artificial viscosity (oracle/av.py) against what the
mathematics fixes: orthonormality of the modal basis (Gauss quadrature),
one-hot modal coefficients of basis functions, the smoothness share of exact
mode mixtures and of a brute-force L2 projection (least squares on a fine
Gauss grid, no Parseval), the values of the switch, eps_0 for a resolved and
for a discontinuous field, and, with the viscosity in the method: uniform
eps acting as extra nu, conservation of the integral, zero eps reducing to
the plain step, and damping of an under-resolved front."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import av
from oracle.element import gll_nodes_weights
from oracle.physics import Burgers, Euler
from oracle.sdc import DGLevel, MLSDC


@pytest.mark.parametrize("P", [2, 5, 8])
def test_modal_basis_is_orthonormal(P):
    xq, wq = npleg.leggauss(P + 3)
    V = av.orthonormal_legendre(P, xq)
    assert np.allclose(V.T @ (wq[:, None] * V), np.eye(P + 1), atol=1e-13)
    for k in range(P + 1):
        c = np.zeros(k + 1)
        c[k] = np.sqrt((2 * k + 1) / 2.0)
        assert np.allclose(V[:, k], npleg.legval(xq, c), atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_basis_functions_have_one_hot_coefficients(dim):
    P = 4
    xg, _ = gll_nodes_weights(P)
    V = av.orthonormal_legendre(P, xg)
    ks = [(1, 3), (4, 0)] if dim == 2 else [(2, 0, 4), (1, 3, 2)]
    for k in ks:  # k = (k_x, k_y[, k_z])
        if dim == 2:
            u = np.einsum("j,i->ji", V[:, k[1]], V[:, k[0]])  # axes (y, x)
        else:
            u = np.einsum("l,j,i->lji", V[:, k[2]], V[:, k[1]], V[:, k[0]])
        c = av.modal_coefficients(P, dim, u.ravel())
        want = np.zeros((P + 1,) * dim)
        want[tuple(reversed(k))] = 1.0
        assert np.allclose(c, want, atol=1e-12)


def _brute_share(P, f):
    """||u - Pi u||^2 / ||u||^2 in 2-D by least squares on a Gauss grid."""
    xq, wq = npleg.leggauss(2 * P + 4)
    X, Y = np.meshgrid(xq, xq, indexing="xy")
    W = np.outer(wq, wq).ravel()
    u = f(X, Y).ravel()
    cols = []
    for a in range(P):
        for b in range(P):
            ca = np.zeros(a + 1)
            ca[a] = 1
            cb = np.zeros(b + 1)
            cb[b] = 1
            cols.append((npleg.legval(X, ca) * npleg.legval(Y, cb)).ravel())
    A = np.stack(cols, axis=1)
    sw = np.sqrt(W)
    coef, *_ = np.linalg.lstsq(A * sw[:, None], u * sw, rcond=None)
    r = u - A @ coef
    return float(np.sum(W * r * r) / np.sum(W * u * u))


@pytest.mark.parametrize("P", [3, 6])
def test_smoothness_share(P):
    xg, _ = gll_nodes_weights(P)
    X, Y = np.meshgrid(xg, xg, indexing="xy")  # arrays (y, x): x fastest
    low = 1.0 + 0.5 * X ** (P - 1) * Y - 0.25 * Y ** (P - 1)
    assert av.smoothness(P, 2, low.ravel()) < 1e-26
    cP = np.zeros(P + 1)
    cP[P] = 1.0
    top = npleg.legval(X, cP)
    assert av.smoothness(P, 2, top.ravel()) == pytest.approx(1.0, rel=1e-12)
    # a mixture of the mean mode and a top mode: share b^2 / (a^2 + b^2) of the
    # orthonormal coefficients
    a, b = 0.8, 0.3
    nP = np.sqrt((2 * P + 1) / 2.0) * np.sqrt(0.5)
    mix = a * 0.5 + b * nP * npleg.legval(Y, cP)  # orthonormal: a L~0 L~0 + b L~0 L~P
    assert av.smoothness(P, 2, mix.ravel()) == pytest.approx(b * b / (a * a + b * b), rel=1e-12)

    def f(x, y):
        return np.tanh(3.0 * x - 1.0) * (1.0 + 0.3 * y * y) + 0.2 * np.sin(2.0 * y)
    # a general polynomial of degree P: the brute-force projection agrees
    coeffs = np.random.default_rng(4).standard_normal((P + 1, P + 1))

    def g(x, y):
        return npleg.legval2d(x, y, coeffs)
    assert av.smoothness(P, 2, g(X, Y).ravel()) == pytest.approx(_brute_share(P, g), rel=1e-10)
    assert f(X, Y).shape == X.shape


def test_switch_values():
    s0, k = -3.0, 0.5
    assert av.switch(s0 - k - 1e-9, s0, k) == 0.0
    assert av.switch(s0 + k + 1e-9, s0, k) == 1.0
    assert av.switch(s0, s0, k) == pytest.approx(0.5, abs=1e-15)
    assert av.switch(s0 + k / 3, s0, k) == pytest.approx(0.75, abs=1e-15)
    assert av.switch(s0 - k, s0, k) == pytest.approx(0.0, abs=1e-15)
    assert av.switch(s0 + k, s0, k) == pytest.approx(1.0, abs=1e-15)
    s = np.linspace(s0 - 2 * k, s0 + 2 * k, 201)
    v = np.array([av.switch(x, s0, k) for x in s])
    assert np.all(np.diff(v) >= 0.0) and np.max(np.abs(np.diff(v))) < 0.03


def test_element_eps_resolved_and_discontinuous():
    ph = Burgers(2, 0.01)
    lv = DGLevel(ph, (4, 3), [0, 0], [1, 1], 6, 3)
    x = lv.coords()
    smooth = (0.5 + 0.3 * np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1]))[None]
    assert np.all(av.element_eps(lv.mesh, ph, smooth, 0.5, 0.5) == 0.0)
    # a jump inside the elements of column 1 (x in [0.25, 0.5])
    step = np.where(x[0] < 0.4, 1.5, 0.5)[None]
    eps = av.element_eps(lv.mesh, ph, step, 0.5, 0.5)
    h = min(1 / 4, 1 / 3)
    for e in range(lv.mesh.E):
        col = e % 4
        if col == 1:
            assert eps[e] == pytest.approx(0.5 * h / 6 * 1.5, rel=1e-14)
        else:
            assert eps[e] == 0.0


def _iso_field(lv, val):
    return np.full(lv.mesh.shape(1)[1:], val)


def test_uniform_eps_acts_as_extra_viscosity():
    nu, c = 0.01, 0.004
    lv = DGLevel(Burgers(2, nu), (3, 2), [0, 0], [1, 1.25], 4, 3)
    ref = DGLevel(Burgers(2, nu + c), (3, 2), [0, 0], [1, 1.25], 4, 3)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(lv.shape())
    lv.av = _iso_field(lv, c)
    assert np.allclose(lv.frhs(u), ref.frhs(u), atol=1e-12)
    assert np.allclose(lv.coef(u, 0.01, None), ref.coef(u, 0.01, None), atol=1e-15)


def test_system_viscosity_conserves_and_is_symmetric():
    ph = Euler(2, 1.4)
    lv = DGLevel(ph, (3, 3), [0, 0], [1, 1], 3, 2)
    rng = np.random.default_rng(3)
    eps = rng.uniform(0.0, 0.01, lv.mesh.E)
    lv.av = av.nodal(lv.mesh, eps)
    rho = 1.0 + 0.1 * rng.standard_normal(lv.shape()[1:])
    U = np.stack([rho, 0.1 * rho, -0.05 * rho, 2.5 + 0.1 * rho])
    F = lv.frhs(U)
    lv2 = DGLevel(ph, (3, 3), [0, 0], [1, 1], 3, 2)
    # the viscosity term moves no mass, momentum or energy: the weak-form
    # right-hand sides (already multiplied by the mass matrix) sum to the
    # same totals with and without it
    dF = (F - lv2.frhs(U)).reshape(4, -1)
    assert np.max(np.abs(dF)) > 1e-6
    assert np.allclose(dF.sum(axis=1), 0.0, atol=1e-13)
    # K_{eps I} is symmetric positive semi-definite (dense, one component)
    n = lv.mesh.E * lv.mesh.Np
    K = np.zeros((n, n))
    e = np.zeros(n)
    Dc = lv._iso(lv.av)
    for j in range(n):
        e[j] = 1.0
        K[:, j] = lv.dg.sipg(Dc, e.reshape((1,) + lv.shape()[1:])).ravel()
        e[j] = 0.0
    assert np.allclose(K, K.T, atol=1e-12)
    assert np.min(np.linalg.eigvalsh(0.5 * (K + K.T))) > -1e-10


def _front_levels(n=6, Ps=(5, 3), Ms=(3, 2), nu=1e-3):
    ph = Burgers(2, nu)
    return ph, [DGLevel(ph, (n, 2), [0, 0], [1, 0.4], P, M, rtol=1e-13) for P, M in zip(Ps, Ms)]


def test_zero_eps_is_the_plain_step_and_mass_is_conserved():
    ph, lv = _front_levels()
    x = lv[0].coords()
    u = (1.0 + 0.5 * np.tanh(np.sin(2 * np.pi * x[0]) / 0.05))[None]
    plain = MLSDC(list(reversed(lv)), n_coarse=2, start="cascade", cycles=2).step(u, 2e-3)
    ph2, lv2 = _front_levels()
    zero = MLSDC(list(reversed(lv2)), n_coarse=2, start="cascade", cycles=2, av=(0.5, 0.0)).step(u, 2e-3)
    assert np.allclose(zero, plain, atol=1e-12)
    ph3, lv3 = _front_levels()
    withav = MLSDC(list(reversed(lv3)), n_coarse=2, start="cascade", cycles=2, av=(0.5, 0.5)).step(u, 2e-3)
    assert lv3[0].dg.integral(withav)[0] == pytest.approx(lv3[0].dg.integral(u)[0], rel=1e-12)
    assert np.max(np.abs(lv3[0].av)) > 0.0


def test_viscosity_damps_an_under_resolved_front():
    x0 = _front_levels()[1][0].coords()
    u0 = (1.0 + 0.5 * np.tanh(np.sin(2 * np.pi * x0[0]) / 0.02))[None]
    out = {}
    for key, avp in (("plain", None), ("av", (2.0, 0.5))):
        ph, lv = _front_levels()
        ml = MLSDC(list(reversed(lv)), n_coarse=2, start="cascade", cycles=2, av=avp)
        u = u0.copy()
        for _ in range(6):
            u = ml.step(u, 2e-3)
        out[key] = u
    # overshoot above the larger state (1.5) and undershoot below the smaller (0.5)
    over = {k: max(np.max(v) - 1.5, 0.5 - np.min(v)) for k, v in out.items()}
    assert over["av"] < 0.6 * over["plain"]


@pytest.mark.parametrize("P,kappa", [(4, 0.5), (6, 2.0)])
def test_switch_centre_is_p_to_the_minus_four(P, kappa):
    """An element whose top-mode share is exactly P^-4 sits at the centre of
    the switch (eps = eps_0 / 2); one at P^-4 10^kappa at its top."""
    ph = Burgers(2, 0.01)
    lv = DGLevel(ph, (1, 1), [0, 0], [2.0, 3.0], P, 2)
    xg, _ = gll_nodes_weights(P)
    V = av.orthonormal_legendre(P, xg)
    for share, frac in ((float(P) ** -4, 0.5), (float(P) ** -4 * 10 ** kappa, 1.0)):
        b = np.sqrt(share)
        a = np.sqrt(1.0 - share)
        u = a * np.outer(V[:, 0], V[:, 0]) + b * np.outer(V[:, 0], V[:, P])  # axes (y, x): top mode in x
        eps = av.element_eps(lv.mesh, ph, u.reshape(lv.shape()), kappa, 0.3)
        eps0 = 0.3 * (2.0 / P) * np.max(np.abs(u))
        assert eps[0] == pytest.approx(frac * eps0, rel=1e-9)
