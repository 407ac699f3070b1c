"""The library's largest shapes against the oracle, through the C ABI:
degree P = 8 on hexahedra (729 nodes per element, the largest element
tile) for the convective operator, f (with the viscous term for
Navier-Stokes), the SIPG and Helmholtz operators and a Helmholtz solve,
for a scalar equation and two systems; M = 8 collocation nodes (the most
the tables take) in a three-level step; and the smallest meshes (one
element along an axis, where an element is its own neighbour)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sdc import DGLevel, MLSDC
from helpers import rel_l2, oracle_phys, lib_problem, random_state, smooth_state

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


@pytest.mark.parametrize("eq,n", [("burgers", (2, 1, 2)), ("euler", (1, 2, 2)), ("ns", (1, 2, 1))])
def test_hexahedra_of_degree_8(S, eq, n):
    dim, P = 3, 8
    lo = [0.0] * dim
    hi = [1.0, 1.25, 1.5]
    phys = oracle_phys(eq, dim)
    lv = DGLevel(phys, n, lo, hi, P, 3, rtol=1e-14)
    sv = S.Solver(lib_problem(S, eq, dim, n, lo, hi), S.make_method([P], [3], cg_rtol=1e-14, cg_maxit=5000))
    rng = np.random.default_rng(8)
    U = random_state(phys, lv.mesh, rng)
    out = torch.empty(U.size, dtype=torch.float64, device="cuda")
    sv.apply(S.OP_CONV, 0, dev(U.ravel()), out)
    assert rel_l2(host(out), lv.conv(U)) < TOL
    sv.apply(S.OP_FRHS, 0, dev(U.ravel()), out)
    assert rel_l2(host(out), lv.frhs(U)) < TOL
    sv.set_state(dev(U.ravel()))
    params = phys.step_params(U)
    if params is not None:
        sv.update_step_params()
    dtm = 0.013
    Dc = lv.coef(U, dtm, params)
    X = rng.standard_normal(lv.shape())
    aux = dev(U[:1].ravel()) if eq == "burgers" else None
    sv.apply(S.OP_SIPG, 0, dev(X.ravel()), out, dt_m=dtm, aux=aux)
    assert rel_l2(host(out), lv.K(Dc, X)) < TOL
    sv.apply(S.OP_HELM, 0, dev(X.ravel()), out, dt_m=dtm, aux=aux)
    assert rel_l2(host(out), lv.dg.helmholtz(Dc, dtm, X)) < TOL
    b = lv.mass(X)
    xo = lv.solve(Dc, dtm, b, np.zeros_like(b))
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    st = sv.helmholtz_solve(0, dtm, dev(b.ravel()), x, coef_state=aux, rtol=1e-14, maxit=5000)
    assert st["converged"]
    assert rel_l2(host(x), xo) < TOL
    sv.close()


def test_eight_nodes_three_levels_and_one_element_axes(S):
    eq, dim, n = "convdiff", 2, (1, 3)
    Ps, Ms = [6, 4, 2], [8, 5, 3]
    lo, hi = [0.0, 0.0], [1.0, 1.25]
    phys = oracle_phys(eq, dim)
    levels = [DGLevel(phys, n, lo, hi, P, M, rtol=1e-14) for P, M in zip(Ps, Ms)]
    meth = S.make_method(Ps, Ms, start=S.START_FMG, n_iter=2, cg_rtol=1e-14, cg_maxit=5000)
    sv = S.Solver(lib_problem(S, eq, dim, n, lo, hi), meth)
    u = smooth_state(phys, levels[0], np.random.default_rng(9))
    ml = MLSDC(list(reversed(levels)), n_coarse=2, start="fmg", cycles=2, post_sweep=True)
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k in range(2):
        st = sv.step(0.02)
        u = ml.step(u, 0.02)
        sv.get_state(out)
        assert rel_l2(host(out), u) < TOL, k
        assert st["not_converged"] == 0
    sv.close()
