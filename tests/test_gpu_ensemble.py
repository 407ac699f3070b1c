"""Stacked ensembles (problem `stack` = B): B independent instances of one
problem in one handle, stacked along the last axis, every kernel launched
once for all of them.  Through the C ABI:
  * each instance's slice of the stacked state after whole steps matches the
    oracle stepping that instance alone at the 1e-12 bar (the stacked
    Helmholtz systems are solved jointly; at the 1e-14 tolerance every
    instance is converged), on the general SIPG path (Burgers, 2-D) and on
    the isotropic paths (IMEX Euler: quadrilaterals, hexahedra, and the
    brick-staged P = 7 hexahedral matvec);
  * the node coordinates of every instance are those of the single problem;
  * at the production tolerance the stacked steps agree with separate
    handles to the tolerance's level;
  * what a stack cannot carry is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sdc import DGLevel, MLSDC
from helpers import rel_l2, oracle_phys, lib_problem, smooth_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18526_amd import sisdc
    return sisdc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _states(phys, lv, B, seed):
    out = []
    for k in range(B):
        u = smooth_state(phys, lv, np.random.default_rng(seed + k))
        out.append(u * (1.0 + 0.2 * k) + 0.1 * k)
    return out


CASES = [
    ("burgers", 2, (3, 4), [6, 3], [4, 3], 3, "si2", 4e-3),
    ("convdiff", 2, (4, 2), [5, 3], [3, 2], 3, "eu", 1e-2),
    ("convdiff", 3, (2, 3, 2), [3, 2], [3, 2], 2, "eu", 1e-2),
    ("convdiff", 3, (2, 2, 2), [7, 3], [3, 2], 2, "eu", 1e-2),
]


@pytest.mark.parametrize("eq,dim,n,Ps,Ms,B,scheme,dt", CASES)
def test_stacked_instances_match_oracle(S, eq, dim, n, Ps, Ms, B, scheme, dt):
    lo = [0.0] * dim
    hi = [1.0 + 0.25 * d for d in range(dim)]
    nu = 5e-3 if eq == "burgers" else 0.02
    phys = oracle_phys(eq, dim, nu=nu)
    integ = S.IMEX_EULER if scheme == "eu" else S.SI2
    meth = S.make_method(Ps, Ms, integrator=integ, start=S.START_CASCADE, n_iter=2, cg_rtol=1e-14, cg_maxit=5000,
                         conserve=0)
    prob = lib_problem(S, eq, dim, n, lo, hi, nu=nu)
    prob.stack = B
    sv = S.Solver(prob, meth)
    E, Np, nv, M = sv.level_info(0)
    levels = [DGLevel(phys, n, lo, hi, P, Mm, rtol=1e-14) for P, Mm in zip(Ps, Ms)]
    Ei = levels[0].mesh.E
    assert E == B * Ei
    # coordinates: every instance on the single problem's box
    xs = sv.coords(0).reshape(dim, B, Ei * Np)
    xo = np.stack([c.reshape(-1) for c in levels[0].coords()])
    for k in range(B):
        assert np.max(np.abs(xs[:, k] - xo)) < 1e-14
    us = _states(phys, levels[0], B, 30)
    sv.set_state(dev(np.concatenate([u.reshape(-1) for u in us])))
    out = torch.empty(B * us[0].size, dtype=torch.float64, device="cuda")
    refs = list(us)
    for step in range(2):
        st = sv.step(dt)
        assert st["not_converged"] == 0
        sv.get_state(out)
        got = out.cpu().numpy().reshape(B, -1)
        for k in range(B):
            lv_k = [DGLevel(phys, n, lo, hi, P, Mm, rtol=1e-14) for P, Mm in zip(Ps, Ms)]
            ml = MLSDC(list(reversed(lv_k)), n_coarse=2, start="cascade", cycles=2, post_sweep=True, scheme=scheme)
            refs[k] = ml.step(refs[k], dt)
            assert rel_l2(got[k], refs[k].reshape(-1)) < 1e-12, (step, k)
    sv.close()


def test_stack_agrees_with_separate_handles_at_production_tolerance(S):
    eq, dim, n, Ps, Ms, B, dt = "burgers", 2, (6, 5), [6, 3], [4, 3], 4, 4e-3
    lo, hi = [0.0, 0.0], [1.0, 1.25]
    phys = oracle_phys(eq, dim, nu=5e-3)
    lv = DGLevel(phys, n, lo, hi, Ps[0], Ms[0])
    us = _states(phys, lv, B, 50)
    meth = S.make_method(Ps, Ms, start=S.START_CASCADE, n_iter=3, cg_rtol=1e-10, cg_maxit=3000, conserve=0)
    prob = lib_problem(S, eq, dim, n, lo, hi, nu=5e-3)
    singles = []
    for k in range(B):
        s1 = S.Solver(prob, meth)
        s1.set_state(dev(us[k].reshape(-1)))
        singles.append(s1)
    prob.stack = B
    sv = S.Solver(prob, meth)
    sv.set_state(dev(np.concatenate([u.reshape(-1) for u in us])))
    out = torch.empty(B * us[0].size, dtype=torch.float64, device="cuda")
    one = torch.empty(us[0].size, dtype=torch.float64, device="cuda")
    for step in range(3):
        sv.step(dt)
        sv.get_state(out)
        got = out.cpu().numpy().reshape(B, -1)
        for k in range(B):
            singles[k].step(dt)
            singles[k].get_state(one)
            assert rel_l2(got[k], one.cpu().numpy()) < 1e-8, (step, k)
    for s1 in singles:
        s1.close()
    sv.close()


def test_what_a_stack_cannot_carry_is_refused(S):
    meth = S.make_method([4, 2], [3, 2], conserve=0)
    prob = S.make_problem(2, (4, 4), (0.0, 0.0), (10.0, 10.0), S.EQ_EULER, stack=2)
    with pytest.raises(S.SisdcError, match="scalar"):
        S.Solver(prob, meth)
    prob = S.make_problem(2, (4, 4), (0.0, 0.0), (1.0, 1.0), S.EQ_BURGERS, nu=0.01, stack=2)
    with pytest.raises(S.SisdcError, match="conserve"):
        S.Solver(prob, S.make_method([4, 2], [3, 2]))
    with pytest.raises(S.SisdcError, match="h_coarsen"):
        S.Solver(prob, S.make_method([4, 2], [3, 2], conserve=0, h_coarsen=[0, 1]))
