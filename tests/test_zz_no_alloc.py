"""helmholtz_solve_noalloc (the solve on the library's fixed per-GPU scratch)
against helmholtz_solve on the same handle and inputs, through the C ABI:
two calls in a row, the second on a smaller level, each compared to the
1e-12 FP64 bar; levels too large for the scratch are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import rel_l2, lib_problem, oracle_phys, random_state
from oracle.sdc import DGLevel

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


@pytest.mark.parametrize("eq,dim,n,Ps", [("burgers", 2, (5, 4), [8, 4]), ("euler", 3, (3, 2, 2), [7, 3]),
                                         ("convdiff", 2, (9, 7), [6, 3])])
def test_noalloc_matches_helmholtz_solve(S, eq, dim, n, Ps):
    lo, hi = [0.0] * dim, [1.0 + 0.25 * d for d in range(dim)]
    phys = oracle_phys(eq, dim)
    prob = lib_problem(S, eq, dim, n, lo, hi)
    meth = S.make_method(Ps, [3, 2], cg_rtol=1e-14, cg_maxit=5000, cg_variant=S.CG_MULTI_KERNEL)
    sv = S.Solver(prob, meth)
    rng = np.random.default_rng(77)
    fine = DGLevel(phys, n, lo, hi, Ps[0], 3)
    Ub = random_state(phys, fine.mesh, rng)
    if phys.system:
        sv.set_state(dev(Ub.ravel()))
        sv.update_step_params()
    coarse_state = torch.empty(sv.level_info(1)[0] * sv.level_info(1)[1] * sv.level_info(1)[2],
                               dtype=torch.float64, device="cuda")
    sv.apply(S.OP_PROJECT, 0, dev(Ub.ravel()), coarse_state)
    for level, dtm in ((0, 0.05), (1, 0.02)):           # the second call is on the smaller level
        E, Np, nv, M = sv.level_info(level)
        b = dev(rng.standard_normal(nv * E * Np))
        ub = (dev(Ub[:1].ravel()) if level == 0 else coarse_state[:E * Np].clone()) if eq == "burgers" else None
        x0 = dev(0.1 * rng.standard_normal(nv * E * Np))
        xa = x0.clone()
        xb = x0.clone()
        sa = sv.helmholtz_solve(level, dtm, b, xa, coef_state=ub, rtol=1e-14, maxit=5000)
        sb = sv.helmholtz_solve_noalloc(level, dtm, b, xb, coef_state=ub, rtol=1e-14, maxit=5000)
        assert sa["converged"] and sb["converged"]
        assert rel_l2(xb.cpu().numpy(), xa.cpu().numpy()) < TOL, (level, sa, sb)
        assert sb["iters"] == sa["iters"]
    sv.close()


def test_noalloc_refuses_levels_beyond_the_scratch(S):
    # 128 x 128 elements at P = 8: 1 327 104 values per vector, 6 vectors (64 MiB) > 32 MiB
    prob = S.make_problem(2, (128, 128), (0.0, 0.0), (1.0, 1.0), S.EQ_CONVDIFF, a=(1.0, 0.5), nu=0.01)
    meth = S.make_method([8], [3], cg_rtol=1e-10, cg_maxit=100)
    sv = S.Solver(prob, meth)
    E, Np, nv, M = sv.level_info(0)
    b = torch.zeros(E * Np, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(S.SisdcError, match="static scratch"):
        sv.helmholtz_solve_noalloc(0, 0.01, b, x)
    sv.close()
