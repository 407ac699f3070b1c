"""Pins of the oracle's Burgers physics: the flux u^2/2, its local
Lax-Friedrichs wave speed |u|, and the semi-implicit coefficient
(dt_m/2) u_b^2 (1,..,1)(1,..,1)^T + nu I.

None of these is fixed by conservation or by a fixed point alone (a flux of
u^2 conserves as well, and the coefficient only moves the iterates), so each
test compares against a result that depends on the exact constant:
  * C(u) against the analytic weak derivative -M div(u^2/2 (1,1)) of a
    resolved smooth field, with spectral decay in P (Sec. 2, eq. burgers);
  * C(c + eps v) against the linear convective operator with velocity
    c (1,1) on a rough field, to O(eps^2): the Jacobian of the Burgers flux at
    c is c and the LLF speed at c is |c| (Sec. 6, the interface flux);
  * one SI(1) / SI(2) substep of the DG Burgers equation linearised about a
    constant state c, on a resolved Fourier mode, against the closed-form
    scalar amplification of Sec. 5 (eq. dahlquist) with A_c = c and
    A_d = nu, i.e. lam_i = -2 pi c (k_x + k_y), lam_r = -nu (2 pi)^2 |k|^2
    and K = (dt/2) lam_i^2 - lam_r (eq. H_SI(1)).
CPU only.
"""
import numpy as np
import pytest

from oracle.element import RefElement
from oracle.mesh import Mesh
from oracle.dg import DG
from oracle.physics import Burgers, ConvDiff
from oracle import sdc


def _dg(phys, n, P, L=1.0):
    ref = RefElement(P)
    mesh = Mesh(n, [0.0] * len(n), [L] * len(n), P)
    return ref, mesh, DG(ref, mesh, phys)


def _smooth(x, y):
    u = 0.4 + 0.3 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.2 * np.cos(2 * np.pi * (x - 2 * y))
    ux = 0.6 * np.pi * np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y) - 0.4 * np.pi * np.sin(2 * np.pi * (x - 2 * y))
    uy = -0.6 * np.pi * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) + 0.8 * np.pi * np.sin(2 * np.pi * (x - 2 * y))
    return u, ux, uy


def test_burgers_conv_is_the_weak_divergence_of_half_u_squared():
    """M^-1 C(u) -> -(u u_x + u u_y) spectrally in P for a smooth periodic u."""
    errs = []
    for P in (4, 6, 8, 10):
        ref, mesh, dg = _dg(Burgers(2, 0.0), (4, 4), P)
        x, y = mesh.node_coords(ref.x)
        u, ux, uy = _smooth(x, y)
        exact = -(u * ux + u * uy)
        got = dg.conv(u[None])[0] / dg.Wm[0]
        errs.append(np.max(np.abs(got - exact)) / np.max(np.abs(exact)))
    assert errs[-1] < 5e-5, errs
    # spectral: every two degrees gain at least a factor 10
    for e1, e2 in zip(errs, errs[1:]):
        assert e2 < 0.1 * e1, errs


@pytest.mark.parametrize("c", [0.8, -0.6])
def test_burgers_llf_flux_linearises_to_upwind_advection(c):
    """Burgers C(c + eps v) = ConvDiff(c (1,1)).C(eps v) + O(eps^2) for a rough
    v (jumps at every face, so the LLF dissipation with speed |c| matters)."""
    n, P = (3, 4), 3
    ref, mesh, dgb = _dg(Burgers(2, 0.0), n, P)
    _, _, dgl = _dg(ConvDiff([c, c], 0.0), n, P)
    rng = np.random.default_rng(11)
    v = rng.standard_normal(mesh.shape(1))
    ratios = []
    for eps in (1e-3, 5e-4):
        lin = dgl.conv(eps * v)
        got = dgb.conv(c + eps * v)
        err = np.max(np.abs(got - lin))
        ratios.append(err / np.max(np.abs(lin)))
    # the remainder is O(eps^2): relative O(eps), halving with eps
    assert ratios[0] < 5e-3, ratios
    assert 1.6 < ratios[0] / ratios[1] < 2.4, ratios


def test_burgers_llf_speed_is_the_larger_absolute_value():
    """For two constant states separated by one face the LLF flux is
    1/2 (f(a) + f(b)) - 1/2 max(|a|, |b|) (b - a) (the a-side view, normal +x):
    1-D-like field in x, checked at the face node weights."""
    n, P = (2, 1), 2
    ref, mesh, dg = _dg(Burgers(2, 0.0), n, P)
    a, b = 0.3, -0.9
    U = np.empty(mesh.shape(1))
    U[0, :, 0] = a          # element e_x = 0
    U[0, :, 1] = b          # element e_x = 1
    C = dg.conv(U)
    # element 0, its +x face (node index P along x), y-face nodes j: weight J_f w_j
    fstar = 0.5 * (0.5 * a * a + 0.5 * b * b) - 0.5 * max(abs(a), abs(b)) * (b - a)
    hy = mesh.h[1]
    wf = 0.5 * hy * ref.w
    # volume term vanishes (constant in the element); the lift at the +x face is -(f* - f(a)) w_f;
    # the -x face of element 0 meets element 1 (periodic) with the mirrored pair
    fstar_left = 0.5 * (0.5 * b * b + 0.5 * a * a) - 0.5 * max(abs(a), abs(b)) * (a - b)
    exp_right = -wf * (fstar - 0.5 * a * a)
    exp_left = -wf * (-fstar_left + 0.5 * a * a)   # outward normal -x: f.n = -f
    got = C[0, 0, 0]                                   # (ey, ex) = (0, 0): shape (iy, ix)
    assert np.allclose(got[:, P], exp_right, rtol=1e-14, atol=1e-15)
    assert np.allclose(got[:, 0], exp_left, rtol=1e-14, atol=1e-15)
    assert np.allclose(got[:, 1:P], 0.0, atol=1e-15)


def _si_amplification(lam_r, lam_i, dt, scheme):
    """One SI substep on the scalar test equation (Sec. 5): mass 1, C -> i lam_i,
    K -> (dt/2) lam_i^2 - lam_r; returns u1 / u0."""
    K = 0.5 * dt * lam_i ** 2 - lam_r
    r1 = (1 + 1j * dt * lam_i) / (1 + dt * K)
    if scheme == "si1":
        return r1
    return (1 + 1j * dt * lam_i * r1) / (1 + dt * K)


@pytest.mark.parametrize("scheme", ["si1", "si2"])
def test_burgers_si_substep_matches_scalar_reduction(scheme):
    """The DG Burgers predictor with one Radau node (one SI substep of length
    dt) applied to u0 = c + eps cos(2 pi k.x): the perturbation moves by the
    scalar amplification with lam_i = -2 pi c (k_x + k_y) (Jacobian of u^2/2
    at c), lam_r = -nu (2 pi)^2 |k|^2 and the SI coefficient
    (dt/2) c^2 (1,1)(1,1)^T + nu I.  dt is chosen so that the implicit
    Lax-Wendroff term is O(1): dropping its factor 1/2 or using u_b instead
    of u_b^2 changes the result at the 1e-1 level."""
    c, nu, eps = 0.7, 0.01, 1e-6
    k = np.array([1.0, 2.0])
    P, n = 10, (4, 4)
    lv = sdc.DGLevel(Burgers(2, nu), n, [0, 0], [1, 1], P, 1, rtol=1e-15, maxit=4000)
    x, y = lv.coords()
    th = 2 * np.pi * (k[0] * x + k[1] * y)
    u0 = (c + eps * np.cos(th))[None]
    lam_i = -2 * np.pi * c * (k[0] + k[1])
    lam_r = -nu * (2 * np.pi) ** 2 * (k @ k)
    dt = 1.2 / abs(lam_i)
    U = sdc.predictor(lv, u0, dt, None, scheme)
    pert = (U[1][0] - c) / eps
    R = _si_amplification(lam_r, lam_i, dt, scheme)
    expect = R.real * np.cos(th) - R.imag * np.sin(th)
    err = np.max(np.abs(pert - expect))
    assert err < 1e-5, err
    # the same check detects a coefficient without the factor 1/2
    K_wrong = dt * lam_i ** 2 - lam_r
    R_wrong = (1 + 1j * dt * lam_i) / (1 + dt * K_wrong)
    assert abs(R_wrong - _si_amplification(lam_r, lam_i, dt, "si1")) > 0.05


def test_burgers_coef_on_fourier_mode():
    """K_{D(c)} cos(2 pi k.x) = M (2 pi)^2 k^T ((dt/2) c^2 11^T + nu I) k cos(...)
    for a constant coefficient state c (the multi-d SI coefficient with the
    Burgers Jacobian f'(c) = c on each axis)."""
    c, nu, dtm = -0.9, 0.004, 0.05
    k = np.array([2.0, 1.0])
    P, n = 10, (4, 4)
    ref, mesh, dg = _dg(Burgers(2, nu), n, P)
    x, y = mesh.node_coords(ref.x)
    X = np.cos(2 * np.pi * (k[0] * x + k[1] * y))[None]
    Dc = Burgers(2, nu).coef(np.full(mesh.shape(1), c), dtm, None)
    Dm = 0.5 * dtm * c * c * np.ones((2, 2)) + nu * np.eye(2)
    lam = (2 * np.pi) ** 2 * (k @ Dm @ k)
    err = np.max(np.abs(dg.sipg(Dc, X) / dg.Wm - lam * X))
    assert err < 1e-6 * lam
