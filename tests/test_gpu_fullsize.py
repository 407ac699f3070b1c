"""Full-size checks at the workloads' own sizes and launch configurations.

* The two-level Burgers workload (32 x 32 elements, P 8/4, M 5/3): one step
  against the oracle, element by element, (a) at a PCG tolerance of 1e-14
  (multi-kernel PCG) to the FP64 bar of 1e-12, and (b) in the configuration
  the bench times (persistent PCG, tolerance 1e-10).  At a relative residual
  of 1e-10 per solve the two sides' solutions differ by up to the
  tolerance times the conditioning of the Helmholtz systems; the step-to-
  step amplification stays O(1), so the bar is 1e-8.
* The 3-D Navier-Stokes workload (16^3, P 7/3) is too large for the oracle:
  one step checks the properties that hold at any size: mass, momentum and
  energy conserved (up to the PCG tolerance: each solve leaves a residual
  whose sum is bounded by rtol |b|), kinetic energy not increasing, state
  finite.
* The 64-instance batch: one batch step, every instance conserving its
  mass to the PCG tolerance, and finite.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sdc import DGLevel, MLSDC
from oracle.physics import Burgers
from helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18526_amd import sisdc
    return sisdc


def totals(S, sv, u):
    """Per-variable totals 1^T M u of a state (device tensor)."""
    E, Np, nv, M = sv.level_info(0)
    mu = torch.empty_like(u)
    sv.apply(S.OP_MASS, 0, u, mu)
    return mu.reshape(nv, -1).sum(dim=1).cpu().numpy()


@pytest.mark.parametrize("config", ["tight_multi", "bench_persistent"])
def test_burgers_workload_step_matches_oracle(S, config):
    from paper_2504_18526_amd.inputs import burgers_field
    from paper_2504_18526_amd.workloads import burgers_2level
    w = burgers_2level()
    rtol = 1e-14 if config == "tight_multi" else w["cg_rtol"]
    variant = S.CG_MULTI_KERNEL if config == "tight_multi" else S.CG_AUTO
    prob = S.make_problem(2, w["n_elem"], w["lo"], w["hi"], S.EQ_BURGERS, nu=w["nu"])
    meth = S.make_method(w["P"], w["M"], start=S.START_CASCADE, n_coarse_sweeps=w["n_coarse"],
                         post_sweep=w["post_sweep"], n_iter=w["cycles"], cg_rtol=rtol, cg_maxit=5000,
                         cg_variant=variant)
    sv = S.Solver(prob, meth)
    E, Np, nv, M = sv.level_info(0)
    x = sv.coords(0)
    u0 = np.ascontiguousarray(burgers_field([x[0], x[1]], seed=w["seed"], kmax=w["kmax"])[None].reshape(nv, E, Np))
    ud = torch.from_numpy(u0.copy()).cuda()
    sv.set_state(ud)
    st = sv.step(w["dt"])
    if config == "bench_persistent":
        assert st["not_converged"] == 0
    out = torch.empty_like(ud)
    sv.get_state(out)
    ph = Burgers(2, w["nu"])
    lv = [DGLevel(ph, w["n_elem"], w["lo"], w["hi"], P, Mm, rtol=rtol) for P, Mm in zip(w["P"], w["M"])]
    ml = MLSDC(list(reversed(lv)), n_coarse=w["n_coarse"], start="cascade", cycles=w["cycles"], post_sweep=True)
    ref = ml.step(u0.reshape(lv[0].shape()), w["dt"])
    got = out.cpu().numpy().reshape(ref.shape)
    bar = 1e-12 if config == "tight_multi" else 1e-8
    assert rel_l2(got, ref) < bar
    # element by element: the worst element is within 100x the global bar
    ge, re = got.reshape(E, Np), ref.reshape(E, Np)
    per = np.linalg.norm(ge - re, axis=1) / np.maximum(np.linalg.norm(re, axis=1), 1e-300)
    assert per.max() < 100 * bar
    sv.close()


def test_ns_workload_step_conserves(S):
    from paper_2504_18526_amd.inputs import taylor_green
    from paper_2504_18526_amd.workloads import ns_2level, systems_dt
    w = ns_2level()
    prob = S.make_problem(3, w["n_elem"], w["lo"], w["hi"], S.EQ_NS, gamma=w["gamma"], mu=w["mu"], Pr=w["Pr"])
    meth = S.make_method(w["P"], w["M"], start=S.START_CASCADE, n_coarse_sweeps=w["n_coarse"],
                         post_sweep=w["post_sweep"], n_iter=w["cycles"], cg_rtol=w["cg_rtol"], cg_maxit=2000)
    sv = S.Solver(prob, meth)
    E, Np, nv, M = sv.level_info(0)
    x = sv.coords(0)
    u0 = np.ascontiguousarray(taylor_green([x[d] for d in range(3)], mach=w["mach"]).reshape(nv, E, Np))
    dt = systems_dt(w, u0)
    ud = torch.from_numpy(u0.copy()).cuda()
    sv.set_state(ud)
    t0 = totals(S, sv, ud)
    st = sv.step(dt)
    assert st["not_converged"] == 0
    out = torch.empty_like(ud)
    sv.get_state(out)
    assert bool(torch.isfinite(out).all())
    t1 = totals(S, sv, out)
    # each solve changes 1^T M u by 1^T (b - A x), |.| <= |1| |r| <= rtol |1| |b| ~ rtol x (the total);
    # a factor 10 covers |b| against the total over the step's solves
    scale = np.array([abs(t0[0]), abs(t0[0]), abs(t0[0]), abs(t0[0]), abs(t0[4])])  # momentum totals are ~0
    bar = 10.0 * st["solves"] * w["cg_rtol"]
    assert np.all(np.abs(t1 - t0) <= bar * scale), (t0, t1, bar)

    def kinetic(u):
        u = u.reshape(nv, E * Np)
        ke = 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0]
        kd = torch.zeros(nv * E * Np, dtype=torch.float64, device="cuda")
        kd[:E * Np] = ke
        md = torch.empty_like(kd)
        sv.apply(S.OP_MASS, 0, kd, md)
        return float(md[:E * Np].sum())

    assert kinetic(out) <= kinetic(ud)
    sv.close()


def test_batch_workload_step_conserves_mass(S):
    from paper_2504_18526_amd.inputs import burgers_field, convdiff_field
    from paper_2504_18526_amd.workloads import batch_instances
    inst = batch_instances(64)
    probs, meths = [], []
    for wi in inst:
        eqc = S.EQ_CONVDIFF if wi["eq"] == "convdiff" else S.EQ_BURGERS
        probs.append(S.make_problem(2, wi["n_elem"], wi["lo"], wi["hi"], eqc, a=wi["a"][:2], nu=wi["nu"]))
        meths.append(S.make_method(wi["P"], wi["M"], start=S.START_CASCADE, n_coarse_sweeps=wi["n_coarse"],
                                   post_sweep=wi["post_sweep"], n_iter=wi["cycles"], cg_rtol=wi["cg_rtol"],
                                   cg_maxit=2000, precision=S.MIXED))
    batch = S.Batch(probs, meths)
    before = []
    for i, wi in enumerate(inst):
        m = batch[i]
        E, Np, nv, M = m.level_info(0)
        x = m.coords(0)
        f = convdiff_field if wi["eq"] == "convdiff" else burgers_field
        u0 = np.ascontiguousarray(f([x[0], x[1]], seed=wi["seed"], kmax=wi["kmax"])[None].reshape(nv, E, Np))
        ud = torch.from_numpy(u0).cuda()
        m.set_state(ud)
        before.append((totals(S, m, ud), float(torch.linalg.norm(ud))))
    stats = batch.step([wi["dt"] for wi in inst])
    for i, wi in enumerate(inst):
        assert stats[i]["not_converged"] == 0, i
        m = batch[i]
        E, Np, nv, M = m.level_info(0)
        out = torch.empty(nv * E * Np, dtype=torch.float64, device="cuda")
        m.get_state(out)
        assert bool(torch.isfinite(out).all()), i
        t0, n0 = before[i]
        t1 = totals(S, m, out)
        # each solve changes 1^T M u by at most |1| rtol |b|, |b| ~ |M u| ~ (area / N) |u| on a unit
        # square: per step <= solves x rtol x |u| / sqrt(N); a factor 10 covers |b| against |M u|
        bar = 10.0 * stats[i]["solves"] * wi["cg_rtol"] * n0 / np.sqrt(E * Np)
        assert abs(t1[0] - t0[0]) <= bar, (i, t0, t1, bar)
    batch.close()
