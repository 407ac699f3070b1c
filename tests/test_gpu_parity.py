"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every stage is fed the same seeded input on both sides and compared by the
relative L2 norm of the difference; the bar for the FP64 path is 1e-12 per
stage.  Meshes are small enough for the oracle, with element counts that
leave a ragged last workgroup (EPB elements per workgroup: 10 at P = 4,
3 at P = 8, 5 at P = 6 in 2-D; 4 at P = 3 in 3-D).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sdc as osdc
from oracle.sdc import DGLevel, SpaceTransfer, SpaceTransferH, MLSDC
from oracle import solve as osolve
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


def make_pair(S, eq, dim, n, Ps, Ms, lo=None, hi=None, nu=0.01, rtol=1e-14, **meth):
    lo = lo if lo is not None else [0.0] * dim
    hi = hi if hi is not None else [1.0 + 0.25 * d for d in range(dim)]
    phys = oracle_phys(eq, dim, nu=nu)
    nodes = "lobatto" if meth.get("nodes", S.NODES_RADAU_RIGHT) == S.NODES_LOBATTO else "radau"
    levels = [DGLevel(phys, n, lo, hi, P, M, rtol=1e-14, nodes=nodes) for P, M in zip(Ps, Ms)]
    prob = lib_problem(S, eq, dim, n, lo, hi, nu=nu)
    m = S.make_method(list(Ps), list(Ms), cg_rtol=rtol, cg_maxit=5000, **meth)
    return phys, levels, S.Solver(prob, m)


# shapes: (eq, dim, n_elem, P)
OPS = [
    ("convdiff", 2, (7, 3), 4),
    ("burgers", 2, (5, 4), 8),
    ("euler", 2, (4, 3), 6),
    ("convdiff", 3, (3, 2, 3), 3),
    ("burgers", 3, (2, 3, 2), 2),
    ("euler", 3, (2, 2, 3), 3),
    ("burgers", 2, (1, 3), 5),
    ("ns", 2, (3, 4), 5),
    ("ns", 3, (2, 3, 2), 4),
    ("ns", 3, (2, 1, 2), 7),
    ("euler", 3, (3, 2, 2), 1),
    ("euler", 2, (3, 2), 8),
    ("ns", 2, (1, 4), 3),
    # more face nodes than nodes per workgroup (the face-task kernels run
    # max(nodes, face nodes) threads), and a last workgroup with empty slots
    ("ns", 3, (2, 2, 3), 2),
    ("ns", 2, (3, 3), 2),
]


@pytest.mark.parametrize("eq,dim,n,P", OPS)
def test_coords_and_conv(S, eq, dim, n, P):
    phys, (lv,), sv = make_pair(S, eq, dim, n, [P], [3])
    xo = np.stack([c.reshape(-1) for c in lv.coords()])
    xl = sv.coords(0).reshape(dim, -1)
    assert np.max(np.abs(xo - xl)) < 1e-14
    rng = np.random.default_rng(10 + P)
    U = random_state(phys, lv.mesh, rng)
    out = torch.empty(U.size, dtype=torch.float64, device="cuda")
    sv.apply(S.OP_CONV, 0, dev(U.ravel()), out)
    assert rel_l2(host(out), lv.conv(U)) < TOL
    sv.apply(S.OP_FRHS, 0, dev(U.ravel()), out)
    assert rel_l2(host(out), lv.frhs(U)) < TOL
    sv.apply(S.OP_MASS, 0, dev(U.ravel()), out)
    assert rel_l2(host(out), lv.mass(U)) < TOL


@pytest.mark.parametrize("eq,dim,n,P", OPS)
def test_sipg_and_helmholtz_apply(S, eq, dim, n, P):
    phys, (lv,), sv = make_pair(S, eq, dim, n, [P], [3])
    rng = np.random.default_rng(20 + P)
    Ub = random_state(phys, lv.mesh, rng)
    X = rng.standard_normal(lv.shape())
    dtm = 0.037
    params = phys.step_params(Ub)
    if params is not None:
        lam = sv.set_state(dev(Ub.ravel())) or sv.update_step_params()
        assert abs(lam - params["lam"]) < 1e-14 * params["lam"]
    Dc = lv.coef(Ub, dtm, params)
    out = torch.empty(X.size, dtype=torch.float64, device="cuda")
    aux = dev(Ub[:1].ravel()) if eq == "burgers" else None
    sv.apply(S.OP_SIPG, 0, dev(X.ravel()), out, dt_m=dtm, aux=aux)
    assert rel_l2(host(out), lv.K(Dc, X)) < TOL
    sv.apply(S.OP_HELM, 0, dev(X.ravel()), out, dt_m=dtm, aux=aux)
    assert rel_l2(host(out), lv.dg.helmholtz(Dc, dtm, X)) < TOL


@pytest.mark.parametrize("eq,dim,n,P", [OPS[5], OPS[10], ("convdiff", 2, (3, 2), 2)])
def test_profile_hooks(S, eq, dim, n, P):
    """The measurement hooks run on levels whose face-trace array is larger
    than a nodal vector (3-D P <= 4, 2-D P <= 2), and leave the operators
    intact."""
    phys, (lv,), sv = make_pair(S, eq, dim, n, [P], [3])
    rng = np.random.default_rng(40 + P)
    U = random_state(phys, lv.mesh, rng)
    sv.set_state(dev(U.ravel()))
    for k in (S.K_SIPG_APPLY, S.K_SIPG_TRACE, S.K_CONV, S.K_CG_UPDATE):
        assert sv.profile_kernel(k, 0, 0.01, reps=3) > 0.0
    torch.cuda.synchronize()
    out = torch.empty(U.size, dtype=torch.float64, device="cuda")
    sv.apply(S.OP_CONV, 0, dev(U.ravel()), out)
    assert rel_l2(host(out), lv.conv(U)) < TOL


@pytest.mark.parametrize("variant", ["auto", "multi"])
@pytest.mark.parametrize("eq,dim,n,P", [OPS[0], OPS[1], OPS[2], OPS[4], OPS[5], OPS[9], OPS[10], OPS[11],
                                        OPS[12]])
def test_helmholtz_solve(S, eq, dim, n, P, variant):
    cgv = S.CG_AUTO if variant == "auto" else S.CG_MULTI_KERNEL
    phys, (lv,), sv = make_pair(S, eq, dim, n, [P], [3], cg_variant=cgv)
    rng = np.random.default_rng(30 + P)
    Ub = random_state(phys, lv.mesh, rng)
    params = phys.step_params(Ub)
    if params is not None:
        sv.set_state(dev(Ub.ravel()))
        sv.update_step_params()
    dtm = 0.05
    Dc = lv.coef(Ub, dtm, params)
    b = rng.standard_normal(lv.shape())
    xo = lv.solve(Dc, dtm, b, np.zeros_like(b))
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    st = sv.helmholtz_solve(0, dtm, dev(b.ravel()), x,
                            coef_state=dev(Ub[:1].ravel()) if eq == "burgers" else None,
                            rtol=1e-14, maxit=5000)
    assert st["converged"]
    assert rel_l2(host(x), xo) < TOL
    # a second solve from the solution converges at once
    st2 = sv.helmholtz_solve(0, dtm, dev(b.ravel()), x,
                             coef_state=dev(Ub[:1].ravel()) if eq == "burgers" else None,
                             rtol=1e-10, maxit=5000)
    assert st2["iters"] <= 1


@pytest.mark.parametrize("dim,n,Pf,Pc", [(2, (3, 2), 8, 4), (2, (2, 3), 6, 4), (3, (2, 1, 2), 7, 3)])
def test_space_transfers(S, dim, n, Pf, Pc):
    phys, (lf, lc), sv = make_pair(S, "convdiff", dim, n, [Pf, Pc], [3, 2])
    tr = SpaceTransfer(lf, lc)
    rng = np.random.default_rng(40)
    Xf = rng.standard_normal(lf.shape())
    Xc = rng.standard_normal(lc.shape())
    oc = torch.empty(Xc.size, dtype=torch.float64, device="cuda")
    of = torch.empty(Xf.size, dtype=torch.float64, device="cuda")
    sv.apply(S.OP_PROJECT, 0, dev(Xf.ravel()), oc)
    assert rel_l2(host(oc), tr.P(Xf)) < TOL
    sv.apply(S.OP_RESTRICT, 0, dev(Xf.ravel()), oc)
    assert rel_l2(host(oc), tr.R(Xf)) < TOL
    sv.apply(S.OP_INTERP, 0, dev(Xc.ravel()), of)
    assert rel_l2(host(of), tr.I(Xc)) < TOL
    # embedded interpolation: P I = identity (Sec. 4 transfer operators)
    sv.apply(S.OP_PROJECT, 0, of, oc)
    assert rel_l2(host(oc), Xc) < 1e-13


def level_array(lv, U):
    return np.concatenate([u.ravel() for u in U])


@pytest.mark.parametrize("eq,dim,n,P,M,scheme", [
    ("convdiff", 2, (7, 3), 4, 3, "si2"),
    ("burgers", 2, (5, 4), 6, 4, "si2"),
    ("burgers", 2, (3, 3), 4, 3, "si1"),
    ("euler", 2, (4, 3), 4, 3, "si2"),
    ("convdiff", 3, (2, 3, 2), 3, 2, "si2"),
])
def test_predictor_and_sweep(S, eq, dim, n, P, M, scheme):
    integ = S.SI2 if scheme == "si2" else S.SI1
    hi = [10.0, 10.0, 10.0][:dim] if eq == "euler" else None
    phys, (lv,), sv = make_pair(S, eq, dim, n, [P], [M], hi=hi, integrator=integ)
    rng = np.random.default_rng(50 + P)
    u0 = smooth_state(phys, lv, rng)
    dt = 0.3 if eq == "euler" else 0.02
    params = phys.step_params(u0)
    sv.set_state(dev(u0.ravel()))
    sv.update_step_params()
    # predictor from u0
    full = np.zeros((M + 1,) + u0.shape)
    full[0] = u0
    sv.set_level(0, dev(full.ravel()))
    sv.predict(0, dt)
    got = torch.empty(full.size, dtype=torch.float64, device="cuda")
    sv.get_level(0, got)
    Uo = osdc.predictor(lv, u0, dt, params, scheme)
    assert rel_l2(host(got), level_array(lv, Uo)) < TOL
    # one sweep with a FAS term g from a perturbed iterate
    Up = [Uo[0]] + [Uo[m] + 1e-3 * rng.standard_normal(u0.shape) * (1 if phys.nv == 1 else u0)
                    for m in range(1, M + 1)]
    g = [None] + [1e-3 * rng.standard_normal(u0.shape) * lv.mass(np.ones_like(u0)) for _ in range(M)]
    sv.set_level(0, dev(level_array(lv, Up)))
    sv.sweep(0, dt, dev(np.concatenate([gm.ravel() for gm in g[1:]])))
    sv.get_level(0, got)
    Uo2 = osdc.sweep(lv, Up, dt, params, g, scheme)
    assert rel_l2(host(got), level_array(lv, Uo2)) < TOL
    # a second sweep reuses the stored f, C and K-terms of the first
    sv.sweep(0, dt)
    sv.get_level(0, got)
    Uo3 = osdc.sweep(lv, Uo2, dt, params, g, scheme)
    assert rel_l2(host(got), level_array(lv, Uo3)) < TOL
    # collocation residual of the result
    res = torch.empty(M * u0.size, dtype=torch.float64, device="cuda")
    sv.collocation_residual(0, dt, res)
    Fo = osdc.collocation_residual(lv, Uo3, dt)
    # the residual is a difference of O(1) terms that cancel to ~1e-6, so
    # its rounding error is measured against the size of the terms (M u_m)
    Fo_flat = np.concatenate([f.ravel() for f in Fo[1:]])
    scale = np.linalg.norm(np.concatenate([lv.mass(Uo3[m]).ravel() for m in range(1, M + 1)]))
    assert np.linalg.norm(host(res) - Fo_flat) / scale < TOL


def test_vcycle_two_levels(S):
    phys, (lf, lc), sv = make_pair(S, "burgers", 2, (4, 3), [6, 3], [4, 2], nu=0.02)
    ml = MLSDC([lc, lf], n_coarse=2)
    rng = np.random.default_rng(60)
    u0 = smooth_state(phys, lf, rng)
    dt = 0.01
    ml.set_initial(u0, None)
    Uf = osdc.predictor(lf, u0, dt, None)
    Uc = osdc.predictor(lc, ml.u0[0], dt, None)
    ml.U[1], ml.U[0] = list(Uf), list(Uc)
    sv.set_state(dev(u0.ravel()))
    sv.set_level(0, dev(level_array(lf, Uf)))
    sv.set_level(1, dev(level_array(lc, Uc)))
    sv.vcycle(0, dt)
    ml.vcycle(1, dt)
    gf = torch.empty(5 * u0.size, dtype=torch.float64, device="cuda")
    gc = torch.empty(3 * ml.U[0][0].size, dtype=torch.float64, device="cuda")
    sv.get_level(0, gf)
    sv.get_level(1, gc)
    assert rel_l2(host(gf), level_array(lf, ml.U[1])) < TOL
    assert rel_l2(host(gc), level_array(lc, ml.U[0])) < TOL
    g = torch.empty(2 * ml.U[0][0].size, dtype=torch.float64, device="cuda")
    sv.get_fas(1, g)
    assert rel_l2(host(g), np.concatenate([x.ravel() for x in ml.g[0][1:]])) < TOL


@pytest.mark.parametrize("variant", ["auto", "multi"])
@pytest.mark.parametrize("case", ["convdiff_sl", "burgers_2l_cascade", "euler_3l_fmg", "convdiff_3d_2l",
                                  "ns_3d_2l"])
def test_steps(S, case, variant):
    if case == "convdiff_sl":
        args = dict(eq="convdiff", dim=2, n=(3, 4), Ps=[4], Ms=[3], n_iter=4)
        dt, nsteps = 1.686e-2, 3
    elif case == "burgers_2l_cascade":
        args = dict(eq="burgers", dim=2, n=(4, 3), Ps=[8, 4], Ms=[5, 3], n_iter=3, nu=5e-3,
                    start=S.START_CASCADE)
        dt, nsteps = 5e-3, 2
    elif case == "euler_3l_fmg":
        args = dict(eq="euler", dim=2, n=(4, 4), Ps=[6, 4, 2], Ms=[5, 3, 2], n_iter=2,
                    start=S.START_FMG, lo=[0, 0], hi=[10, 10])
        dt, nsteps = 0.1, 2
    elif case == "convdiff_3d_2l":
        args = dict(eq="convdiff", dim=3, n=(2, 2, 3), Ps=[3, 2], Ms=[3, 2], n_iter=2,
                    start=S.START_CASCADE)
        dt, nsteps = 0.01, 2
    else:
        args = dict(eq="ns", dim=3, n=(2, 3, 2), Ps=[4, 2], Ms=[3, 2], n_iter=2,
                    start=S.START_CASCADE, lo=[0, 0, 0], hi=[2 * np.pi] * 3)
        dt, nsteps = 4e-3, 2
    eq, dim = args["eq"], args["dim"]
    phys, levels, sv = make_pair(S, eq, dim, args["n"], args["Ps"], args["Ms"], lo=args.get("lo"),
                                 hi=args.get("hi"), nu=args.get("nu", 0.01), n_iter=args["n_iter"],
                                 start=args.get("start", S.START_CASCADE),
                                 cg_variant=S.CG_AUTO if variant == "auto" else S.CG_MULTI_KERNEL)
    fine = levels[0]
    rng = np.random.default_rng(70)
    if eq == "euler":
        from paper_2504_18526_amd.inputs import isentropic_vortex
        u = isentropic_vortex(fine.coords())
    elif eq == "ns":
        from paper_2504_18526_amd.inputs import taylor_green
        u = taylor_green(fine.coords(), mach=0.1)
    else:
        u = smooth_state(phys, fine, rng)
    if len(levels) == 1:
        stepper = lambda v: osdc.sdc_step(fine, v, dt, args["n_iter"])
    else:
        start = {S.START_CASCADE: "cascade", S.START_FMG: "fmg"}[args.get("start", S.START_CASCADE)]
        ml = MLSDC(list(reversed(levels)), n_coarse=2, start=start, cycles=args["n_iter"], post_sweep=True)
        stepper = lambda v: ml.step(v, dt)
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    mass0 = fine.dg.integral(u)
    for k in range(nsteps):
        st = sv.step(dt)
        u = stepper(u)
        sv.get_state(out)
        assert rel_l2(host(out), u) < TOL, (case, k)
        assert st["not_converged"] == 0
    # conservation of every conserved variable
    got = host(out).reshape(u.shape)
    assert np.max(np.abs(fine.dg.integral(got) - mass0)) < 1e-12 * max(1.0, np.max(np.abs(mass0)))


def test_steps_with_changing_dt(S):
    """Time steps of changing size on an isotropic level (pure diffusion,
    multi-kernel PCG): the library forms each inverse Jacobi diagonal once
    per (dt_m, nu) and reuses it, also for a step size seen before."""
    eq, dim, n, P, M, K = "convdiff", 3, (2, 3, 2), 3, 3, 3
    lo, hi = [0.0] * dim, [1.0, 1.25, 1.5]
    a = (0.0, 0.0, 0.0)
    phys = oracle_phys(eq, dim, a=a, nu=0.05)
    lv = DGLevel(phys, n, lo, hi, P, M, rtol=1e-14)
    meth = S.make_method([P], [M], n_iter=K, cg_rtol=1e-14, cg_maxit=5000, cg_variant=S.CG_MULTI_KERNEL)
    sv = S.Solver(lib_problem(S, eq, dim, n, lo, hi, a=a, nu=0.05), meth)
    u = smooth_state(phys, lv, np.random.default_rng(71))
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k, dt in enumerate([0.02, 0.01, 0.02, 0.005, 0.01]):
        st = sv.step(dt)
        u = osdc.sdc_step(lv, u, dt, K)
        sv.get_state(out)
        assert rel_l2(host(out), u) < TOL, (k, dt)
        assert st["not_converged"] == 0
    sv.close()


# ---------------------------------------------------------------- IMEX Euler
@pytest.mark.parametrize("variant", ["auto", "multi"])
@pytest.mark.parametrize("case", ["convdiff_sl", "burgers_2l_cascade", "euler_3l_fmg", "ns_3d_2l"])
def test_imex_euler_steps(S, case, variant):
    """IMEX Euler predictor and sweeps (eqs. H_IMEX, DeltaH_EU): the implicit
    term is the physical diffusion alone (none for systems)."""
    if case == "convdiff_sl":
        args = dict(eq="convdiff", dim=2, n=(3, 4), Ps=[4], Ms=[3], n_iter=4)
        dt, nsteps = 1.0e-2, 3
    elif case == "burgers_2l_cascade":
        args = dict(eq="burgers", dim=2, n=(4, 3), Ps=[8, 4], Ms=[5, 3], n_iter=3, nu=5e-3)
        dt, nsteps = 2e-3, 2
    elif case == "euler_3l_fmg":
        args = dict(eq="euler", dim=2, n=(4, 4), Ps=[6, 4, 2], Ms=[5, 3, 2], n_iter=2, start=S.START_FMG,
                    lo=[0, 0], hi=[10, 10])
        dt, nsteps = 0.01, 2
    else:
        args = dict(eq="ns", dim=3, n=(2, 3, 2), Ps=[4, 2], Ms=[3, 2], n_iter=2, lo=[0, 0, 0], hi=[2 * np.pi] * 3)
        dt, nsteps = 1e-3, 2
    eq, dim = args["eq"], args["dim"]
    start = args.get("start", S.START_CASCADE)
    phys, levels, sv = make_pair(S, eq, dim, args["n"], args["Ps"], args["Ms"], lo=args.get("lo"),
                                 hi=args.get("hi"), nu=args.get("nu", 0.01), n_iter=args["n_iter"], start=start,
                                 integrator=S.IMEX_EULER,
                                 cg_variant=S.CG_AUTO if variant == "auto" else S.CG_MULTI_KERNEL)
    fine = levels[0]
    if eq == "euler":
        from paper_2504_18526_amd.inputs import isentropic_vortex
        u = isentropic_vortex(fine.coords())
    elif eq == "ns":
        from paper_2504_18526_amd.inputs import taylor_green
        u = taylor_green(fine.coords(), mach=0.1)
    else:
        u = smooth_state(phys, fine, np.random.default_rng(71))
    if len(levels) == 1:
        stepper = lambda v: osdc.sdc_step(fine, v, dt, args["n_iter"], "eu")
    else:
        name = {S.START_CASCADE: "cascade", S.START_FMG: "fmg"}[start]
        ml = MLSDC(list(reversed(levels)), scheme="eu", n_coarse=2, start=name, cycles=args["n_iter"],
                   post_sweep=True)
        stepper = lambda v: ml.step(v, dt)
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k in range(nsteps):
        st = sv.step(dt)
        u = stepper(u)
        sv.get_state(out)
        assert rel_l2(host(out), u) < TOL, (case, k)
        assert st["not_converged"] == 0


# ---------------------------------------------------------------- L^2 projection
@pytest.mark.parametrize("case", ["burgers_2l_cascade", "convdiff_3l_fmg", "euler_2l", "ns_3d_2l",
                                  "convdiff_3d_2l"])
def test_l2_projection_steps(S, case):
    """Multilevel steps with the L^2 projection as P_x (Sec. 4): the GPU's
    transfer table against the oracle's, through whole steps.  (The Euler
    case is resolved enough that the projected coarse states keep a
    positive pressure: on the 4 x 4, P 6/4/2 vortex of the other tests the
    L^2 projection to P = 2 undershoots it, and the wave speeds are then
    not defined.)"""
    if case == "burgers_2l_cascade":
        args = dict(eq="burgers", dim=2, n=(4, 3), Ps=[8, 4], Ms=[5, 3], n_iter=3, nu=5e-3, start=S.START_CASCADE)
        dt, nsteps = 5e-3, 2
    elif case == "convdiff_3l_fmg":
        args = dict(eq="convdiff", dim=2, n=(3, 4), Ps=[6, 4, 2], Ms=[5, 3, 2], n_iter=2, start=S.START_FMG)
        dt, nsteps = 1e-2, 2
    elif case == "euler_2l":
        args = dict(eq="euler", dim=2, n=(6, 6), Ps=[6, 3], Ms=[3, 2], n_iter=2, start=S.START_CASCADE,
                    lo=[0, 0], hi=[10, 10])
        dt, nsteps = 0.05, 2
    elif case == "convdiff_3d_2l":
        args = dict(eq="convdiff", dim=3, n=(2, 2, 3), Ps=[3, 2], Ms=[3, 2], n_iter=2, start=S.START_CASCADE)
        dt, nsteps = 0.01, 2
    else:
        args = dict(eq="ns", dim=3, n=(2, 3, 2), Ps=[4, 2], Ms=[3, 2], n_iter=2, start=S.START_CASCADE,
                    lo=[0, 0, 0], hi=[2 * np.pi] * 3)
        dt, nsteps = 4e-3, 2
    eq, dim = args["eq"], args["dim"]
    phys, levels, sv = make_pair(S, eq, dim, args["n"], args["Ps"], args["Ms"], lo=args.get("lo"),
                                 hi=args.get("hi"), nu=args.get("nu", 0.01), n_iter=args["n_iter"],
                                 start=args["start"], projection=S.PROJ_L2)
    fine = levels[0]
    if eq == "euler":
        from paper_2504_18526_amd.inputs import isentropic_vortex
        u = isentropic_vortex(fine.coords())
    elif eq == "ns":
        from paper_2504_18526_amd.inputs import taylor_green
        u = taylor_green(fine.coords(), mach=0.1)
    else:
        u = smooth_state(phys, fine, np.random.default_rng(72))
    name = {S.START_CASCADE: "cascade", S.START_FMG: "fmg"}[args["start"]]
    ml = MLSDC(list(reversed(levels)), n_coarse=2, start=name, cycles=args["n_iter"], post_sweep=True,
               projection="l2")
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k in range(nsteps):
        st = sv.step(dt)
        u = ml.step(u, dt)
        sv.get_state(out)
        assert rel_l2(host(out), u) < TOL, (case, k)
        assert st["not_converged"] == 0
    # the coarse initial value is the L^2 projection of the fine one: it has the same integral
    E, Np, nv, M = sv.level_info(1)
    gc = torch.empty((M + 1) * nv * E * Np, dtype=torch.float64, device="cuda")
    sv.get_level(1, gc)
    uc0 = host(gc)[: nv * E * Np].reshape(levels[1].shape())
    np.testing.assert_allclose(levels[1].dg.integral(uc0), fine.dg.integral(host(out).reshape(u.shape)),
                               rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- non-incremental MLSDC
@pytest.mark.parametrize("case", ["burgers_2l_cascade", "convdiff_3l_fmg", "euler_3l_fmg", "ns_3d_2l"])
def test_nonincremental_steps(S, case):
    """Zero-to-node MLSDC (Sec. 4): the library's cumulated time restriction
    against the oracle's literal zero-to-node sweeps, residuals and FAS
    terms.  The result differs from the node-to-node form's (the two are not
    equivalent), by far more than the tolerance."""
    if case == "burgers_2l_cascade":
        args = dict(eq="burgers", dim=2, n=(4, 3), Ps=[8, 4], Ms=[5, 3], n_iter=2, nu=5e-3, start=S.START_CASCADE)
        dt = 5e-3
    elif case == "convdiff_3l_fmg":
        args = dict(eq="convdiff", dim=2, n=(3, 4), Ps=[6, 4, 2], Ms=[5, 3, 2], n_iter=1, start=S.START_FMG)
        dt = 2e-2
    elif case == "euler_3l_fmg":
        args = dict(eq="euler", dim=2, n=(4, 4), Ps=[6, 4, 2], Ms=[5, 3, 2], n_iter=1, start=S.START_FMG,
                    lo=[0, 0], hi=[10, 10])
        dt = 0.1
    else:
        args = dict(eq="ns", dim=3, n=(2, 3, 2), Ps=[4, 2], Ms=[3, 2], n_iter=1, start=S.START_CASCADE,
                    lo=[0, 0, 0], hi=[2 * np.pi] * 3)
        dt = 4e-3
    eq, dim = args["eq"], args["dim"]
    name = {S.START_CASCADE: "cascade", S.START_FMG: "fmg"}[args["start"]]
    res = {}
    for form in ("nonincremental", "incremental"):
        phys, levels, sv = make_pair(S, eq, dim, args["n"], args["Ps"], args["Ms"], lo=args.get("lo"),
                                     hi=args.get("hi"), nu=args.get("nu", 0.01), n_iter=args["n_iter"],
                                     start=args["start"],
                                     formulation=S.NONINCREMENTAL if form == "nonincremental" else S.INCREMENTAL)
        fine = levels[0]
        if eq == "euler":
            from paper_2504_18526_amd.inputs import isentropic_vortex
            u = isentropic_vortex(fine.coords())
        elif eq == "ns":
            from paper_2504_18526_amd.inputs import taylor_green
            u = taylor_green(fine.coords(), mach=0.1)
        else:
            u = smooth_state(phys, fine, np.random.default_rng(73))
        ml = MLSDC(list(reversed(levels)), n_coarse=2, start=name, cycles=args["n_iter"], post_sweep=True,
                   formulation=form)
        sv.set_state(dev(u.ravel()))
        out = torch.empty(u.size, dtype=torch.float64, device="cuda")
        st = sv.step(dt)
        ref = ml.step(u, dt)
        sv.get_state(out)
        assert st["not_converged"] == 0
        assert rel_l2(host(out), ref) < TOL, (case, form)
        res[form] = host(out)
        sv.close()
    assert rel_l2(res["nonincremental"], res["incremental"]) > 1e3 * TOL, case


# ---------------------------------------------------------------- Lobatto nodes
@pytest.mark.parametrize("case", ["convdiff_sl", "burgers_2l_cascade", "euler_3l_fmg", "ns_3d_2l"])
def test_lobatto_steps(S, case):
    """Lobatto collocation nodes (Sec. 3): tau_1 = 0, so the first substep
    is empty and u_1 = u_0."""
    if case == "convdiff_sl":
        args = dict(eq="convdiff", dim=2, n=(3, 4), Ps=[4], Ms=[3], n_iter=4, start=S.START_CASCADE)
        dt, nsteps = 1.0e-2, 2
    elif case == "burgers_2l_cascade":
        args = dict(eq="burgers", dim=2, n=(4, 3), Ps=[8, 4], Ms=[5, 3], n_iter=3, nu=5e-3, start=S.START_CASCADE)
        dt, nsteps = 5e-3, 2
    elif case == "euler_3l_fmg":
        args = dict(eq="euler", dim=2, n=(4, 4), Ps=[6, 4, 2], Ms=[5, 3, 2], n_iter=2, start=S.START_FMG,
                    lo=[0, 0], hi=[10, 10])
        dt, nsteps = 0.1, 2
    else:
        args = dict(eq="ns", dim=3, n=(2, 3, 2), Ps=[4, 2], Ms=[3, 2], n_iter=2, start=S.START_CASCADE,
                    lo=[0, 0, 0], hi=[2 * np.pi] * 3)
        dt, nsteps = 4e-3, 2
    eq, dim = args["eq"], args["dim"]
    phys, levels, sv = make_pair(S, eq, dim, args["n"], args["Ps"], args["Ms"], lo=args.get("lo"),
                                 hi=args.get("hi"), nu=args.get("nu", 0.01), n_iter=args["n_iter"],
                                 start=args["start"], nodes=S.NODES_LOBATTO)
    fine = levels[0]
    if eq == "euler":
        from paper_2504_18526_amd.inputs import isentropic_vortex
        u = isentropic_vortex(fine.coords())
    elif eq == "ns":
        from paper_2504_18526_amd.inputs import taylor_green
        u = taylor_green(fine.coords(), mach=0.1)
    else:
        u = smooth_state(phys, fine, np.random.default_rng(74))
    if len(levels) == 1:
        stepper = lambda v: osdc.sdc_step(fine, v, dt, args["n_iter"])
    else:
        name = {S.START_CASCADE: "cascade", S.START_FMG: "fmg"}[args["start"]]
        ml = MLSDC(list(reversed(levels)), n_coarse=2, start=name, cycles=args["n_iter"], post_sweep=True)
        stepper = lambda v: ml.step(v, dt)
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k in range(nsteps):
        st = sv.step(dt)
        u = stepper(u)
        sv.get_state(out)
        assert rel_l2(host(out), u) < TOL, (case, k)
        assert st["not_converged"] == 0
    # the first collocation node is t_0: the fine level's u_1 is the step's initial value (to rounding:
    # the empty first substep solves M x = M u_0, and the multilevel corrections at that node vanish)
    E, Np, nv, M = sv.level_info(0)
    lvl = torch.empty((M + 1) * nv * E * Np, dtype=torch.float64, device="cuda")
    sv.get_level(0, lvl)
    a = host(lvl).reshape(M + 1, -1)
    np.testing.assert_allclose(a[1], a[0], rtol=1e-14, atol=1e-14 * np.max(np.abs(a[0])))


def test_lobatto_needs_two_nodes(S):
    prob = lib_problem(S, "convdiff", 2, (2, 2), [0.0, 0.0], [1.0, 1.0], nu=0.01)
    with pytest.raises(S.SisdcError, match="Lobatto"):
        S.Solver(prob, S.make_method([4, 2], [3, 1], nodes=S.NODES_LOBATTO))


@pytest.mark.parametrize("nodes", ["radau", "lobatto"])
@pytest.mark.parametrize("M", [2, 3, 5, 8])
def test_node_quadrature(S, M, nodes):
    """q_m = dt sum_i w^nn_{m,i} f_i for all m (eq. nn_weights), host and device buffers."""
    nd = S.NODES_LOBATTO if nodes == "lobatto" else S.NODES_RADAU_RIGHT
    phys, (lv,), sv = make_pair(S, "burgers", 2, (3, 2), [4], [M], nodes=nd)
    rng = np.random.default_rng(60 + M)
    F = [None] + [rng.standard_normal(lv.shape()) for _ in range(M)]
    dt = 0.037
    ref = osdc.quadrature(lv, F, dt)
    f = np.concatenate([F[i].ravel() for i in range(1, M + 1)])
    got_d = torch.empty(f.size, dtype=torch.float64, device="cuda")
    sv.apply(S.OP_QUAD, 0, dev(f), got_d, dt_m=dt)
    got_h = np.empty(f.size)
    sv.apply(S.OP_QUAD, 0, f, got_h, dt_m=dt)
    want = np.concatenate([ref[m].ravel() for m in range(1, M + 1)])
    assert rel_l2(host(got_d), want) < TOL
    assert np.array_equal(host(got_d), got_h)


# ---------------------------------------------------------------- 2:1 h-coarsening
def make_pair_h(S, eq, dim, n, Ps, Ms, hc, lo=None, hi=None, nu=0.01, **meth):
    """Levels whose element counts halve where hc[l] = 1 (h_coarsen)."""
    lo = lo if lo is not None else [0.0] * dim
    hi = hi if hi is not None else [1.0 + 0.25 * d for d in range(dim)]
    phys = oracle_phys(eq, dim, nu=nu)
    ns, cur = [], list(n)
    for l in range(len(Ps)):
        if hc[l]:
            cur = [v // 2 for v in cur]
        ns.append(tuple(cur))
    levels = [DGLevel(phys, nl, lo, hi, P, M, rtol=1e-14) for nl, P, M in zip(ns, Ps, Ms)]
    prob = lib_problem(S, eq, dim, n, lo, hi, nu=nu)
    m = S.make_method(list(Ps), list(Ms), cg_rtol=1e-14, cg_maxit=5000, h_coarsen=list(hc), **meth)
    return phys, levels, S.Solver(prob, m)


@pytest.mark.parametrize("dim,n,Pf,Pc,proj", [(2, (4, 6), 8, 4, "interp"), (2, (4, 2), 5, 5, "interp"),
                                              (2, (6, 4), 6, 3, "l2"), (3, (2, 4, 2), 4, 2, "interp"),
                                              (3, (2, 2, 4), 6, 6, "l2")])
def test_h_transfers(S, dim, n, Pf, Pc, proj):
    phys, (lf, lc), sv = make_pair_h(S, "convdiff", dim, n, [Pf, Pc], [3, 2], [0, 1],
                                     projection=S.PROJ_L2 if proj == "l2" else S.PROJ_INTERP)
    E, Np, nv, M = sv.level_info(1)
    assert E == lc.mesh.E
    tr = SpaceTransferH(lf, lc, proj)
    rng = np.random.default_rng(41)
    Xf = rng.standard_normal(lf.shape())
    Xc = rng.standard_normal(lc.shape())
    oc = torch.empty(Xc.size, dtype=torch.float64, device="cuda")
    of = torch.empty(Xf.size, dtype=torch.float64, device="cuda")
    sv.apply(S.OP_PROJECT, 0, dev(Xf.ravel()), oc)
    assert rel_l2(host(oc), tr.P(Xf)) < TOL
    sv.apply(S.OP_RESTRICT, 0, dev(Xf.ravel()), oc)
    assert rel_l2(host(oc), tr.R(Xf)) < TOL
    sv.apply(S.OP_INTERP, 0, dev(Xc.ravel()), of)
    assert rel_l2(host(of), tr.I(Xc)) < TOL


@pytest.mark.parametrize("case", ["burgers_2l", "convdiff_2l_h_only", "euler_3l_fmg", "ns_3d_2l"])
def test_h_coarsened_steps(S, case):
    """Multilevel steps with 2:1 h-coarsening (and p-coarsening on top)."""
    if case == "burgers_2l":
        args = dict(eq="burgers", dim=2, n=(4, 4), Ps=[8, 4], Ms=[5, 3], hc=[0, 1], n_iter=3, nu=5e-3,
                    start=S.START_CASCADE)
        dt = 5e-3
    elif case == "convdiff_2l_h_only":
        args = dict(eq="convdiff", dim=2, n=(4, 6), Ps=[4, 4], Ms=[3, 3], hc=[0, 1], n_iter=3, start=S.START_CASCADE)
        dt = 1e-2
    elif case == "euler_3l_fmg":
        args = dict(eq="euler", dim=2, n=(8, 8), Ps=[4, 4, 2], Ms=[5, 3, 2], hc=[0, 1, 0], n_iter=2,
                    start=S.START_FMG, lo=[0, 0], hi=[10, 10])
        dt = 0.05
    else:
        args = dict(eq="ns", dim=3, n=(2, 4, 2), Ps=[4, 2], Ms=[3, 2], hc=[0, 1], n_iter=2, start=S.START_CASCADE,
                    lo=[0, 0, 0], hi=[2 * np.pi] * 3)
        dt = 4e-3
    eq, dim = args["eq"], args["dim"]
    phys, levels, sv = make_pair_h(S, eq, dim, args["n"], args["Ps"], args["Ms"], args["hc"], lo=args.get("lo"),
                                   hi=args.get("hi"), nu=args.get("nu", 0.01), n_iter=args["n_iter"],
                                   start=args["start"])
    fine = levels[0]
    if eq == "euler":
        from paper_2504_18526_amd.inputs import isentropic_vortex
        u = isentropic_vortex(fine.coords())
    elif eq == "ns":
        from paper_2504_18526_amd.inputs import taylor_green
        u = taylor_green(fine.coords(), mach=0.1)
    else:
        u = smooth_state(phys, fine, np.random.default_rng(75))
    name = {S.START_CASCADE: "cascade", S.START_FMG: "fmg"}[args["start"]]
    ml = MLSDC(list(reversed(levels)), n_coarse=2, start=name, cycles=args["n_iter"], post_sweep=True)
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k in range(2):
        st = sv.step(dt)
        u = ml.step(u, dt)
        sv.get_state(out)
        assert rel_l2(host(out), u) < TOL, (case, k)
        assert st["not_converged"] == 0


def test_h_coarsening_validation(S):
    prob = lib_problem(S, "convdiff", 2, (3, 4), [0.0, 0.0], [1.0, 1.0], nu=0.01)
    with pytest.raises(S.SisdcError, match="even"):
        S.Solver(prob, S.make_method([4, 2], [3, 2], h_coarsen=[0, 1]))
    prob = lib_problem(S, "convdiff", 3, (2, 2, 2), [0.0] * 3, [1.0] * 3, nu=0.01)
    with pytest.raises(S.SisdcError, match="degrees up to 6"):
        S.Solver(prob, S.make_method([7, 3], [3, 2], h_coarsen=[0, 1]))


# ---------------------------------------------------------------- options together
@pytest.mark.parametrize("scheme", ["si2", "eu"])
def test_all_method_options_together(S, scheme):
    """Lobatto nodes, the zero-to-node form, the L^2 projection and 2:1
    h-coarsening on top of p-coarsening, all in one three-level FMG run."""
    dim, n, Ps, Ms, hc = 2, (8, 4), [5, 4, 2], [4, 3, 2], [0, 1, 0]
    lo, hi, nu, dt = [0.0, 0.0], [1.0, 1.25], 0.01, 1e-2
    phys = oracle_phys("burgers", dim, nu=nu)
    ns, cur = [], list(n)
    for l in range(3):
        if hc[l]:
            cur = [v // 2 for v in cur]
        ns.append(tuple(cur))
    levels = [DGLevel(phys, nl, lo, hi, P, M, rtol=1e-14, nodes="lobatto") for nl, P, M in zip(ns, Ps, Ms)]
    prob = lib_problem(S, "burgers", dim, n, lo, hi, nu=nu)
    m = S.make_method(Ps, Ms, start=S.START_FMG, n_iter=2, cg_rtol=1e-14, cg_maxit=5000, h_coarsen=hc,
                      nodes=S.NODES_LOBATTO, formulation=S.NONINCREMENTAL, projection=S.PROJ_L2,
                      integrator=S.IMEX_EULER if scheme == "eu" else S.SI2)
    sv = S.Solver(prob, m)
    u = smooth_state(phys, levels[0], np.random.default_rng(76))
    ml = MLSDC(list(reversed(levels)), scheme=scheme, n_coarse=2, start="fmg", cycles=2, post_sweep=True,
               projection="l2", formulation="nonincremental")
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k in range(2):
        st = sv.step(dt)
        u = ml.step(u, dt)
        sv.get_state(out)
        assert rel_l2(host(out), u) < TOL, (scheme, k)
        assert st["not_converged"] == 0


# ---------------------------------------------------------------- persistent PCG
# The one-launch pipelined PCG runs at production tolerances (rtol >= 1e-11).
# Its iterates differ from the oracle's exact solve by at most about
# cond(A) * rtol, so the checks here are (i) the TRUE residual of the GPU
# solution, recomputed with the oracle's operator, meets rtol, and (ii) whole
# steps agree with the oracle to 1e-8 (rtol 1e-10 times a condition number of
# the mass-scaled Helmholtz operator below 100 at these sizes).
RTOL_PROD = 1e-10


def launch_variant(S, launch):
    return S.CG_AUTO if launch == "ordinary" else S.CG_PERSISTENT_COOPERATIVE


@pytest.mark.parametrize("launch", ["ordinary", "cooperative"])
@pytest.mark.parametrize("eq,dim,n,P", [OPS[0], OPS[1], OPS[2], OPS[3], OPS[6]])
def test_persistent_solve_true_residual(S, eq, dim, n, P, launch):
    phys, (lv,), sv = make_pair(S, eq, dim, n, [P], [3], rtol=RTOL_PROD, cg_variant=launch_variant(S, launch))
    rng = np.random.default_rng(80 + P)
    Ub = random_state(phys, lv.mesh, rng)
    params = phys.step_params(Ub)
    if params is not None:
        sv.set_state(dev(Ub.ravel()))
        sv.update_step_params()
    dtm = 0.05
    Dc = lv.coef(Ub, dtm, params)
    b = rng.standard_normal(lv.shape())
    x0 = 0.1 * rng.standard_normal(lv.shape())
    x = dev(x0.ravel())
    st = sv.helmholtz_solve(0, dtm, dev(b.ravel()), x,
                            coef_state=dev(Ub[:1].ravel()) if eq == "burgers" else None,
                            rtol=RTOL_PROD, maxit=2000)
    assert st["converged"] and st["iters"] > 0
    xg = host(x).reshape(b.shape)
    res = b - lv.dg.helmholtz(Dc, dtm, xg)
    assert np.linalg.norm(res) <= 1.0001 * RTOL_PROD * np.linalg.norm(b)
    xo = lv.solve(Dc, dtm, b, np.zeros_like(b))
    assert rel_l2(xg, xo) < 1e-8


@pytest.mark.parametrize("launch", ["ordinary", "cooperative"])
@pytest.mark.parametrize("case", ["burgers_2l", "convdiff_1l"])
def test_persistent_steps(S, case, launch):
    cgv = launch_variant(S, launch)
    if case == "burgers_2l":
        phys, levels, sv = make_pair(S, "burgers", 2, (5, 4), [8, 4], [5, 3], nu=5e-3, rtol=RTOL_PROD,
                                     n_iter=3, start=S.START_CASCADE, cg_variant=cgv)
        ml = MLSDC(list(reversed(levels)), n_coarse=2, start="cascade", cycles=3, post_sweep=True)
        dt = 2e-3
        stepper = lambda v: ml.step(v, dt)
    else:
        phys, levels, sv = make_pair(S, "convdiff", 2, (7, 3), [4], [3], rtol=RTOL_PROD, n_iter=4, cg_variant=cgv)
        dt = 1.5e-2
        stepper = lambda v: osdc.sdc_step(levels[0], v, dt, 4)
    fine = levels[0]
    u = smooth_state(phys, fine, np.random.default_rng(90))
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k in range(2):
        st = sv.step(dt)
        assert st["not_converged"] == 0 and st["cg_iters"] > 0
        assert st["max_rel_residual"] <= RTOL_PROD * 1.0001
        u = stepper(u)
        sv.get_state(out)
        assert rel_l2(host(out), u) < 1e-8, (case, k)


def test_persistent_solves_of_two_streams(S):
    """Two handles on two streams, stepped from two host threads at once: the
    library orders their persistent solves on the device, so neither one's
    barrier waits for workgroups the other keeps off the device, and each
    result equals that of the same handle stepped alone (deterministic
    reductions: bit for bit)."""
    import threading
    streams = [torch.cuda.Stream() for _ in range(2)]
    w = [dict(n=(16, 16), P=[8, 4], M=[5, 3], dt=2e-3), dict(n=(24, 20), P=[6, 3], M=[4, 3], dt=2e-3)]
    solvers, u0 = [], []
    for i, c in enumerate(w):
        phys = oracle_phys("burgers", 2, nu=5e-3)
        lv = DGLevel(phys, c["n"], [0.0, 0.0], [1.0, 1.25], c["P"][0], c["M"][0], rtol=1e-14)
        u0.append(smooth_state(phys, lv, np.random.default_rng(300 + i)).ravel())
        prob = lib_problem(S, "burgers", 2, c["n"], [0.0, 0.0], [1.0, 1.25], nu=5e-3)
        m = S.make_method(c["P"], c["M"], start=S.START_CASCADE, n_iter=3, cg_rtol=RTOL_PROD, cg_maxit=2000)
        solvers.append([S.Solver(prob, m, stream=streams[i].cuda_stream) for _ in range(2)])
    for i in range(2):
        for sv in solvers[i]:
            sv.set_state(dev(u0[i]))
    torch.cuda.synchronize()
    errors = []

    def run(i):
        try:
            for _ in range(3):
                st = solvers[i][0].step(w[i]["dt"])
                assert st["not_converged"] == 0
        except Exception as e:  # reported by the main thread
            errors.append((i, e))

    th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for i in range(2):  # the same steps, one handle at a time
        for _ in range(3):
            solvers[i][1].step(w[i]["dt"])
    for i in range(2):
        a = torch.empty(u0[i].size, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        solvers[i][0].get_state(a)
        solvers[i][1].get_state(b)
        assert torch.equal(a, b), i
    for pair in solvers:
        for sv in pair:
            sv.close()


# ---------------------------------------------------------------- mixed precision
# FP32 inner PCG inside FP64 iterative refinement.  With the outer FP64
# residual driven to 1e-12 the result must match the FP64 oracle to 1e-10
# relative L2 per solve and per step (the bar for the mixed form).
RTOL_MIXED = 1e-12


@pytest.mark.parametrize("eq,dim,n,P", [OPS[0], OPS[1], OPS[2], OPS[3], OPS[5], OPS[9], OPS[11]])
def test_mixed_solve(S, eq, dim, n, P):
    phys, (lv,), sv = make_pair(S, eq, dim, n, [P], [3], rtol=RTOL_MIXED, precision=S.MIXED)
    rng = np.random.default_rng(100 + P)
    Ub = random_state(phys, lv.mesh, rng)
    params = phys.step_params(Ub)
    if params is not None:
        sv.set_state(dev(Ub.ravel()))
        sv.update_step_params()
    dtm = 0.05
    Dc = lv.coef(Ub, dtm, params)
    b = rng.standard_normal(lv.shape())
    x = dev(np.zeros(b.size))
    st = sv.helmholtz_solve(0, dtm, dev(b.ravel()), x,
                            coef_state=dev(Ub[:1].ravel()) if eq == "burgers" else None,
                            rtol=RTOL_MIXED, maxit=4000)
    assert st["converged"]
    xg = host(x).reshape(b.shape)
    res = b - lv.dg.helmholtz(Dc, dtm, xg)
    assert np.linalg.norm(res) <= 1.0001 * RTOL_MIXED * np.linalg.norm(b)
    xo = lv.solve(Dc, dtm, b, np.zeros_like(b))
    assert rel_l2(xg, xo) < 1e-10


@pytest.mark.parametrize("case", ["convdiff_sl", "burgers_2l_cascade", "euler_3l_fmg"])
def test_mixed_steps(S, case):
    if case == "convdiff_sl":
        args = dict(eq="convdiff", dim=2, n=(3, 4), Ps=[4], Ms=[3], n_iter=4)
        dt = 1.686e-2
    elif case == "burgers_2l_cascade":
        args = dict(eq="burgers", dim=2, n=(4, 3), Ps=[8, 4], Ms=[5, 3], n_iter=3, nu=5e-3,
                    start=S.START_CASCADE)
        dt = 5e-3
    else:
        args = dict(eq="euler", dim=2, n=(4, 4), Ps=[6, 4, 2], Ms=[5, 3, 2], n_iter=2,
                    start=S.START_FMG, lo=[0, 0], hi=[10, 10])
        dt = 0.1
    eq, dim = args["eq"], args["dim"]
    phys, levels, sv = make_pair(S, eq, dim, args["n"], args["Ps"], args["Ms"], lo=args.get("lo"),
                                 hi=args.get("hi"), nu=args.get("nu", 0.01), n_iter=args["n_iter"],
                                 start=args.get("start", S.START_CASCADE), rtol=RTOL_MIXED,
                                 precision=S.MIXED)
    fine = levels[0]
    if eq == "euler":
        from paper_2504_18526_amd.inputs import isentropic_vortex
        u = isentropic_vortex(fine.coords())
    else:
        u = smooth_state(phys, fine, np.random.default_rng(110))
    if len(levels) == 1:
        stepper = lambda v: osdc.sdc_step(fine, v, dt, args["n_iter"])
    else:
        start = {S.START_CASCADE: "cascade", S.START_FMG: "fmg"}[args["start"]]
        ml = MLSDC(list(reversed(levels)), n_coarse=2, start=start, cycles=args["n_iter"], post_sweep=True)
        stepper = lambda v: ml.step(v, dt)
    sv.set_state(dev(u.ravel()))
    out = torch.empty(u.size, dtype=torch.float64, device="cuda")
    for k in range(2):
        st = sv.step(dt)
        assert st["not_converged"] == 0 and st["ir_rounds"] >= st["solves"]
        u = stepper(u)
        sv.get_state(out)
        assert rel_l2(host(out), u) < 1e-10, (case, k)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("variant", ["auto", "multi"])
@pytest.mark.parametrize("eq,dim,n,P", [OPS[1], OPS[9]])
def test_zero_rhs_solve(S, eq, dim, n, P, variant, precision):
    """Degenerate solve: b = 0 from x0 = 0 returns x = 0 without iterating."""
    cgv = S.CG_AUTO if variant == "auto" else S.CG_MULTI_KERNEL
    prec = S.FP64 if precision == "fp64" else S.MIXED
    phys, (lv,), sv = make_pair(S, eq, dim, n, [P], [3], cg_variant=cgv, precision=prec)
    rng = np.random.default_rng(50 + P)
    Ub = random_state(phys, lv.mesh, rng)
    if phys.step_params(Ub) is not None:
        sv.set_state(dev(Ub.ravel()))
        sv.update_step_params()
    b = np.zeros(lv.shape())
    x = dev(np.zeros(b.size))
    st = sv.helmholtz_solve(0, 0.05, dev(b.ravel()), x,
                            coef_state=dev(Ub[:1].ravel()) if eq == "burgers" else None, rtol=1e-10, maxit=100)
    assert st["converged"]
    assert st["iters"] == 0
    assert float(torch.abs(x).max()) == 0.0


@pytest.mark.parametrize("eq,dim,n,Ps,Ms", [("convdiff", 2, (3, 2), [4, 2], [3, 2]),
                                             ("burgers", 2, (2, 3), [5, 3], [4, 2]),
                                             ("euler", 2, (3, 3), [4], [3]),
                                             ("ns", 3, (2, 1, 2), [3, 2], [3, 2])])
def test_constant_state_is_steady(S, eq, dim, n, Ps, Ms):
    """A constant state is an exact steady solution of every equation (all
    fluxes constant, all jumps zero): one full step leaves it unchanged."""
    phys, levels, sv = make_pair(S, eq, dim, n, Ps, Ms, rtol=1e-12, n_iter=2)
    fine = levels[0]
    shp = fine.shape()
    if phys.nv == 1:
        U = np.full(shp, 0.7)
    else:
        U = np.empty(shp)
        rho, v, p = 1.3, [0.2, -0.1, 0.05][:dim], 0.9
        U[0] = rho
        for k in range(dim):
            U[1 + k] = rho * v[k]
        U[dim + 1] = p / (phys.gamma - 1.0) + 0.5 * rho * sum(vk * vk for vk in v)
    sv.set_state(dev(U.ravel()))
    sv.step(1e-3 if dim == 2 else 5e-4)
    out = torch.empty(U.size, dtype=torch.float64, device="cuda")
    sv.get_state(out)
    assert rel_l2(host(out), U) < 1e-13
