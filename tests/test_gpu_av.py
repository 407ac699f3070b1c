"""GPU parity of the Persson-Peraire artificial viscosity (method av_kappa,
av_c) with the oracle (oracle/av.py, oracle/sdc.py), through the C ABI:
  * the element viscosity eps_e from states with fronts (scalar and system,
    2-D and 3-D; elements on and off the switch);
  * F(u) and the implicit operator K_D, M + dt_m K_D with eps_e in the
    diffusion, at the 1e-12 bar;
  * whole two-level steps (the viscosity evaluated from u_0 at the start of
    each step) at the 1e-12 bar;
  * the method options that cannot carry it are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import av as oav
from oracle.sdc import DGLevel, MLSDC
from helpers import rel_l2, oracle_phys, lib_problem

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18526_amd import sisdc
    return sisdc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.cpu().numpy()


def front_state(phys, lv, width, seed):
    """A front across x (tanh of the given width) on a smooth background."""
    x = lv.coords()
    dim = lv.mesh.dim
    L0 = lv.mesh.hi[0] - lv.mesh.lo[0]
    xc = lv.mesh.lo[0] + 0.43 * L0
    rng = np.random.default_rng(seed)
    bg = 0.05 * np.sin(2 * np.pi * x[1] / (lv.mesh.hi[1] - lv.mesh.lo[1]) + rng.uniform(0, 6))
    front = np.tanh((x[0] - xc) / width)
    if phys.nv == 1:
        return (1.0 + 0.5 * front + bg)[None]
    rho = 1.0 + 0.4 * front + bg
    vel = [0.1 * np.ones_like(rho) * (d + 1) / dim for d in range(dim)]
    p = np.ones_like(rho)
    E = p / (phys.gamma - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho] + [rho * v for v in vel] + [E])


CASES = [("burgers", 2, (5, 3), 6, (0.5, 0.5)), ("convdiff", 2, (6, 2), 4, (1.0, 0.5)),
         ("euler", 2, (5, 3), 5, (2.0, 0.4)), ("ns", 3, (4, 2, 2), 3, (2.0, 0.4)),
         ("burgers", 3, (4, 2, 3), 4, (0.5, 0.5))]


def _pair(S, eq, dim, n, Ps, Ms, avp, **meth):
    lo = [0.0] * dim
    hi = [1.0 + 0.25 * d for d in range(dim)]
    phys = oracle_phys(eq, dim)
    levels = [DGLevel(phys, n, lo, hi, P, M, rtol=1e-14) for P, M in zip(Ps, Ms)]
    m = S.make_method(list(Ps), list(Ms), cg_rtol=1e-14, cg_maxit=5000, av=avp, **meth)
    return phys, levels, S.Solver(lib_problem(S, eq, dim, n, lo, hi), m)


@pytest.mark.parametrize("eq,dim,n,P,avp", CASES)
def test_element_viscosity_matches_oracle(S, eq, dim, n, P, avp):
    phys, (lv,), sv = _pair(S, eq, dim, n, [P], [3], avp)
    U = front_state(phys, lv, 0.6 * float(np.min(lv.mesh.h)) / P, 5 + P)
    sv.set_state(dev(U.ravel()))
    sv.av_update()
    got = host(sv.av_get(torch.empty(lv.mesh.E, dtype=torch.float64, device="cuda")))
    want = oav.element_eps(lv.mesh, phys, U, *avp)
    assert np.count_nonzero(want) > 0 and np.count_nonzero(want) < lv.mesh.E
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(want)
    sv.close()


@pytest.mark.parametrize("eq,dim,n,P,avp", CASES)
def test_operators_with_viscosity_match_oracle(S, eq, dim, n, P, avp):
    phys, (lv,), sv = _pair(S, eq, dim, n, [P], [3], avp)
    U = front_state(phys, lv, 0.6 * float(np.min(lv.mesh.h)) / P, 7 + P)
    sv.set_state(dev(U.ravel()))
    sv.av_update()
    params = phys.step_params(U)
    if params is not None:
        sv.update_step_params()
    lv.av = oav.nodal(lv.mesh, oav.element_eps(lv.mesh, phys, U, *avp))
    out = torch.empty(U.size, dtype=torch.float64, device="cuda")
    sv.apply(S.OP_FRHS, 0, dev(U.ravel()), out)
    assert rel_l2(host(out), lv.frhs(U)) < TOL
    rng = np.random.default_rng(3)
    X = rng.standard_normal(lv.shape())
    dtm = 0.021
    Dc = lv.coef(U, dtm, params)
    aux = dev(U[:1].ravel()) if eq == "burgers" else None
    sv.apply(S.OP_SIPG, 0, dev(X.ravel()), out, dt_m=dtm, aux=aux)
    assert rel_l2(host(out), lv.K(Dc, X)) < TOL
    sv.apply(S.OP_HELM, 0, dev(X.ravel()), out, dt_m=dtm, aux=aux)
    assert rel_l2(host(out), lv.dg.helmholtz(Dc, dtm, X)) < TOL
    sv.close()


@pytest.mark.parametrize("eq,dim,n,Ps,Ms,dt,avp", [
    ("burgers", 2, (6, 2), [5, 3], [3, 2], 2e-3, (2.0, 0.5)),
    ("euler", 2, (5, 2), [4, 2], [3, 2], 4e-3, (2.0, 0.4)),
    ("convdiff", 2, (4, 3), [6, 3], [4, 3], 1e-2, (1.0, 0.5)),
])
def test_steps_with_viscosity_match_oracle(S, eq, dim, n, Ps, Ms, dt, avp):
    phys, levels, sv = _pair(S, eq, dim, n, Ps, Ms, avp, start=S.START_CASCADE, n_iter=2)
    U = front_state(phys, levels[0], 0.5 * float(np.min(levels[0].mesh.h)) / Ps[0], 11)
    ml = MLSDC(list(reversed(levels)), n_coarse=2, start="cascade", cycles=2, post_sweep=True, av=avp)
    sv.set_state(dev(U.ravel()))
    out = torch.empty(U.size, dtype=torch.float64, device="cuda")
    ref = U
    for k in range(2):
        st = sv.step(dt)
        ref = ml.step(ref, dt)
        sv.get_state(out)
        assert rel_l2(host(out), ref) < TOL, k
        assert st["not_converged"] == 0
    assert np.count_nonzero(levels[0].av) > 0
    sv.close()


def test_methods_that_cannot_carry_viscosity_are_refused(S):
    prob = S.make_problem(2, (4, 4), (0.0, 0.0), (1.0, 1.0), S.EQ_BURGERS, nu=0.01)
    for kw, msg in ((dict(precision=S.MIXED), "FP64"), (dict(h_coarsen=[0, 1]), "same elements")):
        with pytest.raises(S.SisdcError, match=msg):
            S.Solver(prob, S.make_method([4, 2], [3, 2], av=(0.5, 0.5), **kw))
    with pytest.raises(S.SisdcError, match="av_kappa"):
        S.Solver(prob, S.make_method([4, 2], [3, 2], av=(0.0, 0.5)))
    sv = S.Solver(prob, S.make_method([4, 2], [3, 2]))
    with pytest.raises(S.SisdcError, match="no artificial viscosity"):
        sv.av_update()
    sv.close()
