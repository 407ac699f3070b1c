"""Failure handling through the C ABI, forced from the host so every kernel
still ends normally:
  * an iteration cap too small for the tolerance: SISDC_ENOTCONV, with the
    statistics written and the handle usable afterwards;
  * a non-finite value in the initial state: SISDC_ENONFINITE (persistent,
    multi-kernel and mixed-precision solves);
  * mixed-precision refinement that stalls (an inner tolerance that barely
    lowers the residual): FP64 PCG finishes the solve, counted in
    ir_fallbacks, and the step still matches plain FP64 to the 1e-10 bar."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sdc import DGLevel
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


def _solver(S, eq, dim, n, Ps, Ms, **meth):
    lo, hi = [0.0] * dim, [1.0 + 0.25 * d for d in range(dim)]
    if eq == "euler":
        lo, hi = [0.0] * dim, [10.0] * dim
    phys = oracle_phys(eq, dim)
    fine = DGLevel(phys, n, lo, hi, Ps[0], Ms[0])
    sv = S.Solver(lib_problem(S, eq, dim, n, lo, hi), S.make_method(Ps, Ms, **meth))
    if eq == "euler":
        from paper_2504_18526_amd.inputs import isentropic_vortex
        u = isentropic_vortex(fine.coords())
    else:
        u = smooth_state(phys, fine, np.random.default_rng(5))
    return sv, u


@pytest.mark.parametrize("variant", ["auto", "multi"])
@pytest.mark.parametrize("eq,dim,n,Ps,Ms", [("burgers", 2, (4, 3), [8, 4], [5, 3]),
                                            ("euler", 2, (3, 3), [4, 2], [3, 2])])
def test_iteration_cap_reports_enotconv(S, eq, dim, n, Ps, Ms, variant):
    cgv = S.CG_AUTO if variant == "auto" else S.CG_MULTI_KERNEL
    sv, u = _solver(S, eq, dim, n, Ps, Ms, cg_rtol=1e-10, cg_maxit=1, cg_variant=cgv, n_iter=1)
    sv.set_state(dev(u.ravel()))
    st = S.Stats()
    rc = sv._lib.sisdc_step(sv.h, 0.0, 0.01 if eq == "burgers" else 0.05, ctypes.byref(st))
    assert rc == S.ENOTCONV, sv._lib.sisdc_last_error().decode()
    assert "cg_maxit" in sv._lib.sisdc_last_error().decode()
    assert st.not_converged > 0 and st.solves >= st.not_converged
    assert st.cg_iters_max <= 1
    # a direct solve with the same cap: ENOTCONV, the iterate written
    E, Np, nv, M = sv.level_info(0)
    b = dev(np.random.default_rng(1).standard_normal(nv * E * Np))
    x = torch.zeros_like(b)
    ub = dev(u[:1].ravel()) if eq == "burgers" else None
    with pytest.raises(S.SisdcError) as ei:
        sv.helmholtz_solve(0, 0.01, b, x, coef_state=ub, rtol=1e-12, maxit=1)
    assert ei.value.code == S.ENOTCONV
    assert float(torch.linalg.norm(x)) > 0.0
    # the handle still works with an adequate cap
    sv2, _ = _solver(S, eq, dim, n, Ps, Ms, cg_rtol=1e-10, cg_maxit=2000, cg_variant=cgv, n_iter=1)
    sv2.set_state(dev(u.ravel()))
    st2 = sv2.step(0.01 if eq == "burgers" else 0.05)
    assert st2["not_converged"] == 0
    sv.close()
    sv2.close()


@pytest.mark.parametrize("eq,variant,precision", [("convdiff", "auto", "fp64"), ("burgers", "multi", "fp64"),
                                                  ("euler", "multi", "fp64"), ("burgers", "auto", "mixed")])
def test_nonfinite_state_reports_enonfinite(S, eq, variant, precision):
    cgv = S.CG_AUTO if variant == "auto" else S.CG_MULTI_KERNEL
    prec = S.MIXED if precision == "mixed" else S.FP64
    dim, n, Ps, Ms = 2, (3, 3), [4, 2], [3, 2]
    sv, u = _solver(S, eq, dim, n, Ps, Ms, cg_rtol=1e-10, cg_maxit=200, cg_variant=cgv, precision=prec, n_iter=1)
    u = u.copy()
    u.reshape(-1)[7] = np.nan
    sv.set_state(dev(u.ravel()))
    with pytest.raises(S.SisdcError) as ei:
        sv.step(0.01)
    assert ei.value.code == S.ENONFINITE, str(ei.value)
    # a finite state afterwards steps normally on the same handle
    u.reshape(-1)[7] = 0.5 if eq != "euler" else u.reshape(-1)[8]
    sv.set_state(dev(u.ravel()))
    assert sv.step(0.01)["not_converged"] == 0
    sv.close()


def test_stalled_refinement_falls_back_to_fp64(S):
    eq, dim, n, Ps, Ms = "burgers", 2, (4, 3), [6, 3], [3, 2]
    dt = 5e-3
    plain, u = _solver(S, eq, dim, n, Ps, Ms, cg_rtol=1e-12, cg_maxit=4000, n_iter=2)
    # each FP32 inner solve only has to lower its residual by 10 %: the FP64
    # residual then shrinks too slowly and refinement is declared stalled
    mixed, _ = _solver(S, eq, dim, n, Ps, Ms, cg_rtol=1e-12, cg_maxit=4000, n_iter=2, precision=S.MIXED,
                       inner_rtol=0.9)
    ref = torch.empty(u.size, dtype=torch.float64, device="cuda")
    got = torch.empty_like(ref)
    plain.set_state(dev(u.ravel()))
    mixed.set_state(dev(u.ravel()))
    plain.step(dt)
    st = mixed.step(dt)
    plain.get_state(ref)
    mixed.get_state(got)
    assert st["ir_fallbacks"] > 0
    assert st["not_converged"] == 0
    assert rel_l2(got.cpu().numpy(), ref.cpu().numpy()) < 1e-10
    plain.close()
    mixed.close()
