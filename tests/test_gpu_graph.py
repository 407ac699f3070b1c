"""Step graphs (sisdc_set_graph, sisdc_batch_set_graph) through the C ABI.

A captured step replays the kernels of the uncaptured step in the same order
(every persistent PCG solve still stops on its own device-side test), so a
replayed step must equal the uncaptured step bit for bit.  Replays are
checked one by one, with the program's own eager work (state reads, direct
Helmholtz solves on the same handle, which use the same tagged records) and
synchronisations between them; another dt captures again; forms that need
the host inside a step run uncaptured."""
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


def _pair(S, eq, n, Ps, Ms, nu=0.01, **meth):
    lo, hi = [0.0, 0.0], [1.0, 1.25]
    m = S.make_method(Ps, Ms, start=S.START_CASCADE, n_iter=2, cg_rtol=1e-10, cg_maxit=3000, **meth)
    a = S.Solver(lib_problem(S, eq, 2, n, lo, hi, nu=nu), m)
    b = S.Solver(lib_problem(S, eq, 2, n, lo, hi, nu=nu), m)
    phys = oracle_phys(eq, 2, nu=nu)
    levels = [DGLevel(phys, n, lo, hi, P, M, rtol=1e-14) for P, M in zip(Ps, Ms)]
    u = smooth_state(phys, levels[0], np.random.default_rng(7))
    return a, b, phys, levels, u


def _state(sv, n):
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    sv.get_state(out)
    return out.cpu().numpy()


@pytest.mark.parametrize("eq,n,Ps,Ms", [("convdiff", (4, 3), [6, 3], [4, 3]), ("burgers", (5, 4), [8, 4], [5, 3])])
def test_replayed_steps_equal_uncaptured_steps(S, eq, n, Ps, Ms):
    g, plain, phys, levels, u = _pair(S, eq, n, Ps, Ms, nu=5e-3 if eq == "burgers" else 0.01)
    g.set_graph(True)
    g.set_state(dev(u.ravel()))
    plain.set_state(dev(u.ravel()))
    dt = 4e-3 if eq == "burgers" else 1e-2
    ref = u.copy()
    rng = np.random.default_rng(3)
    E, Np, nv, M = g.level_info(0)
    for k in range(4):
        st = g.step(dt)
        sp = plain.step(dt)
        last, caps, reps = g.graph_info()
        assert last and caps == 1 and reps == k + 1
        assert st["solves"] == sp["solves"] and st["cg_iters"] == sp["cg_iters"]
        assert st["fine_sweeps"] == sp["fine_sweeps"] and st["not_converged"] == 0
        got, want = _state(g, u.size), _state(plain, u.size)
        assert np.array_equal(got, want), k
        # eager work on the same handle between replays: a direct solve (its
        # persistent launch uses the tagged records the graph also uses)
        b = rng.standard_normal(nv * E * Np)
        x1, x2 = torch.zeros(b.size, dtype=torch.float64, device="cuda"), None
        x2 = torch.zeros_like(x1)
        cs = dev(got[:E * Np]) if eq == "burgers" else None
        s1 = g.helmholtz_solve(0, dt / M, dev(b), x1, coef_state=cs, rtol=1e-10, maxit=3000)
        s2 = plain.helmholtz_solve(0, dt / M, dev(b), x2, coef_state=cs, rtol=1e-10, maxit=3000)
        assert s1["converged"] and torch.equal(x1, x2)
        ml = MLSDC(list(reversed(levels)), n_coarse=2, start="cascade", cycles=2, post_sweep=True)
        ref = ml.step(ref, dt)
        assert rel_l2(got, ref) < 1e-8, k
    # another step size captures again
    st = g.step(0.5 * dt)
    plain.step(0.5 * dt)
    last, caps, reps = g.graph_info()
    assert last and caps == 2 and reps == 5
    assert np.array_equal(_state(g, u.size), _state(plain, u.size))
    # switching off: uncaptured again
    g.set_graph(False)
    g.step(dt)
    plain.step(dt)
    assert not g.graph_info()[0]
    assert np.array_equal(_state(g, u.size), _state(plain, u.size))
    g.close()
    plain.close()


@pytest.mark.parametrize("why", ["mixed", "tolerance", "system"])
def test_steps_that_need_the_host_run_uncaptured(S, why):
    if why == "system":
        lo, hi = [0.0, 0.0], [10.0, 10.0]
        m = S.make_method([4, 2], [3, 2], start=S.START_CASCADE, n_iter=2, cg_rtol=1e-10, cg_maxit=3000)
        g = S.Solver(lib_problem(S, "euler", 2, (3, 3), lo, hi), m)
        plain = S.Solver(lib_problem(S, "euler", 2, (3, 3), lo, hi), m)
        from paper_2504_18526_amd.inputs import isentropic_vortex
        u = isentropic_vortex(DGLevel(oracle_phys("euler", 2), (3, 3), lo, hi, 4, 3).coords())
        dt = 0.05
    else:
        kw = {"precision": S.MIXED} if why == "mixed" else {}
        g, plain, phys, levels, u = _pair(S, "burgers", (4, 3), [6, 3], [3, 2], nu=5e-3, **kw)
        if why == "tolerance":
            for sv in (g, plain):
                sv.close()
            m = S.make_method([6, 3], [3, 2], start=S.START_CASCADE, n_iter=2, cg_rtol=1e-13, cg_maxit=3000)
            lo, hi = [0.0, 0.0], [1.0, 1.25]
            g = S.Solver(lib_problem(S, "burgers", 2, (4, 3), lo, hi, nu=5e-3), m)
            plain = S.Solver(lib_problem(S, "burgers", 2, (4, 3), lo, hi, nu=5e-3), m)
        dt = 4e-3
    g.set_graph(True)
    g.set_state(dev(u.ravel()))
    plain.set_state(dev(u.ravel()))
    for k in range(2):
        g.step(dt)
        plain.step(dt)
        assert g.graph_info() == (False, 0, 0)
        assert np.array_equal(_state(g, u.size), _state(plain, u.size)), (why, k)
    g.close()
    plain.close()


def test_batch_with_graphs_matches_single_handles(S):
    INST = [("convdiff", (3, 4), 4, 3, 0.02, 1.0e-2), ("burgers", (4, 3), 6, 4, 5e-3, 4.0e-3),
            ("convdiff", (2, 5), 3, 5, 0.05, 8.0e-3), ("burgers", (5, 2), 8, 3, 1e-2, 3.0e-3),
            ("convdiff", (1, 3), 5, 4, 0.01, 1.2e-2), ("burgers", (3, 3), 5, 3, 2e-2, 5.0e-3)]
    probs, meths, us, dts, singles = [], [], [], [], []
    for i, (eq, n, P, M, nu, dt) in enumerate(INST):
        Ps, Ms = [P, (P + 1) // 2], [M, M // 2 + 1]
        lo, hi = [0.0, 0.0], [1.0, 1.25]
        prob = lib_problem(S, eq, 2, n, lo, hi, nu=nu)
        meth = S.make_method(Ps, Ms, start=S.START_CASCADE, n_iter=2, cg_rtol=1e-10, cg_maxit=3000)
        probs.append(prob)
        meths.append(meth)
        phys = oracle_phys(eq, 2, nu=nu)
        us.append(smooth_state(phys, DGLevel(phys, n, lo, hi, P, M), np.random.default_rng(200 + i)))
        dts.append(dt)
        singles.append(S.Solver(prob, meth))
    batch = S.Batch(probs, meths)
    batch.set_threads(3)
    batch.set_graph(True)
    for i, u in enumerate(us):
        batch[i].set_state(dev(u.ravel()))
        singles[i].set_state(dev(u.ravel()))
    for k in range(3):
        batch.step(dts)
        for i in range(len(INST)):
            singles[i].step(dts[i])
            last, caps, reps = batch[i].graph_info()
            assert last and caps == 1 and reps == k + 1, i
            assert np.array_equal(_state(batch[i], us[i].size), _state(singles[i], us[i].size)), (k, i)
    for s in singles:
        s.close()
    batch.close()
