"""GPU checks of the learned-guess MLP against the CPU oracle (oracle/mlp.py)
and the measured effect of the trained network on the PCG solves."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp as omlp
from oracle import sdc as osdc
from helpers import rel_l2, oracle_phys, lib_problem, smooth_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18526_amd import sisdc
    return sisdc


def small_solver(S, P=4, n=(5, 3), rtol=1e-10, n_iter=4):
    prob = lib_problem(S, "convdiff", 2, n, [0, 0], [1, 1])
    meth = S.make_method([P], [3], n_iter=n_iter, cg_rtol=rtol, cg_maxit=2000)
    return S.Solver(prob, meth)


def test_net_init_matches_oracle(S):
    sv = small_solver(S)
    n, H = 25, 24
    sv.net_init(0, H, seed=5, max_batch=128, max_rows=0)
    got = sv.net_params(0)
    ref = omlp.init_params(n, H, seed=5).astype(np.float32)
    assert np.array_equal(got, ref)


def _random_net(S, sv, n, H, seed):
    rng = np.random.default_rng(seed)
    th = (omlp.init_params(n, H, seed) + 0.05 * rng.standard_normal(omlp.n_params(n, H))).astype(np.float32)
    sv.net_set_params(0, th)
    return th, rng


# (P, H): n = (P + 1)^2 inputs.  n = 25 stages operands one value at a time;
# n = 16 and 64 with H = 40 and 136 take the four-wide staging (K % 4 == 0),
# with ragged M, N and K tails (H = 136: two BF16 K slabs of 128, three FP32
# slabs of 64, the last partial).
@pytest.mark.parametrize("P,H", [(4, 40), (3, 40), (7, 136)])
@pytest.mark.parametrize("rows", [1, 37, 100, 257])
def test_forward_fp32_and_bf16(S, rows, P, H):
    sv = small_solver(S, P=P)
    n = (P + 1) ** 2
    sv.net_init(0, H, seed=1, max_batch=512, max_rows=0)
    th, rng = _random_net(S, sv, n, H, 11)
    X = rng.standard_normal((rows, n)).astype(np.float32)
    Y = np.empty((rows, n), dtype=np.float32)
    sv.net_forward(0, X, Y)
    y64, _ = omlp.forward(th.astype(np.float64), X.astype(np.float64), n, H)
    assert rel_l2(Y, y64) < 1e-5
    sv.net_forward(0, X, Y, bf16=True)
    yb, _ = omlp.forward(th, X, n, H, dtype=np.float32, bf16_weights=True)
    # same bfloat16 operands; FP32 accumulation order differs, which can move
    # an intermediate across a bfloat16 rounding boundary now and then
    assert rel_l2(Y, yb) < 2e-3
    assert rel_l2(Y, y64) < 3e-2


@pytest.mark.parametrize("rows,P", [(7, 4), (64, 4), (200, 4), (200, 3)])
def test_gradient_matches_oracle(S, rows, P):
    sv = small_solver(S, P=P)
    n, H = (P + 1) ** 2, 32
    sv.net_init(0, H, seed=2, max_batch=256, max_rows=0)
    th, rng = _random_net(S, sv, n, H, 12)
    X = rng.standard_normal((rows, n)).astype(np.float32)
    T = rng.standard_normal((rows, n)).astype(np.float32)
    G = np.empty(omlp.n_params(n, H), dtype=np.float32)
    loss = sv.net_grad(0, X, T, G)
    L64, g64 = omlp.loss_and_grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64), n, H)
    assert abs(loss - L64) < 1e-5 * L64
    assert rel_l2(G, g64) < 1e-5


def test_adam_step_matches_oracle(S):
    sv = small_solver(S)
    n, H = 25, 16
    sv.net_init(0, H, seed=3, max_batch=64, max_rows=0)
    th, rng = _random_net(S, sv, n, H, 13)
    X = rng.standard_normal((50, n)).astype(np.float32)
    T = rng.standard_normal((50, n)).astype(np.float32)
    opt = omlp.Adam(th.size, lr=1e-3, dtype=np.float32)
    cur = th.copy()
    for k in range(3):
        sv.net_set_params(0, cur)
        G = np.empty_like(cur)
        sv.net_grad(0, X, T, G)
        sv.net_set_params(0, cur)
        sv.net_train_step(0, X, T, 1e-3)
        got = sv.net_params(0)
        ref = opt.step(cur, G)       # the oracle's Adam fed the GPU's gradient
        assert np.max(np.abs(got - ref)) < 1e-6, k
        cur = got


def test_learned_guess_gain(S):
    """Harvest (r0, x* - x0) rows from plain solves, train, then run the same
    steps with and without the network from the same state.  Both reach the
    same tolerance; the test reports the iteration counts and requires the
    results to agree to the solver tolerance and the network not to cost
    iterations."""
    sv = small_solver(S, P=4, n=(8, 8), rtol=1e-10, n_iter=4)
    lv = osdc.DGLevel(oracle_phys("convdiff", 2), (8, 8), [0, 0], [1, 1], 4, 3)
    u = smooth_state(lv.phys, lv, np.random.default_rng(3))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dt = 1.686e-2
    sv.set_state(dev(u.ravel()))
    sv.net_init(0, 64, seed=1, max_batch=1024, max_rows=20000)
    sv.net_harvest(0, 1)
    for _ in range(6):
        sv.step(dt)
    rows = sv.net_harvest(0, 0)
    assert rows > 1000
    loss0 = sv.net_train(0, 1, 256, 1e-3)
    loss = sv.net_train(0, 150, 256, 1e-3)
    assert loss < loss0
    start = torch.empty(u.size, dtype=torch.float64, device="cuda")
    sv.get_state(start)
    out_a = torch.empty_like(start)
    out_b = torch.empty_like(start)
    its = {}
    for use, out in ((False, out_a), (True, out_b)):
        sv.set_state(start)
        sv.net_use(0, use)
        tot = 0
        rej = 0
        for _ in range(3):
            st = sv.step(dt)
            tot += st["cg_iters"]
            rej += st["net_rejected"]
        sv.get_state(out)
        its[use] = (tot, rej)
    print(f"learned guess: CG iterations without {its[False][0]}, with {its[True][0]} "
          f"(rejected guesses {its[True][1]}), train loss {loss0:.3e} -> {loss:.3e}")
    assert rel_l2(out_b.cpu().numpy(), out_a.cpu().numpy()) < 1e-8
    assert its[True][0] <= its[False][0]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["convdiff_1l", "burgers_2l", "ns_3d_2l"])
def test_learned_forms_match_oracle(S, case, precision):
    """The learned initial guess (and the learned guess with mixed-precision
    refinement) changes only the starting point of each PCG solve: every step
    matches the FP64 oracle's step from the same state to the 1e-10 bar
    (GPU PCG tolerance 1e-12, oracle 1e-14).  The network of every level is
    first trained on rows harvested from the GPU's own plain solves."""
    from oracle.sdc import DGLevel, MLSDC, sdc_step
    if case == "convdiff_1l":
        eq, dim, n, Ps, Ms, dt, lo, hi = "convdiff", 2, (6, 5), [4], [3], 1.686e-2, [0, 0], [1, 1]
    elif case == "burgers_2l":
        eq, dim, n, Ps, Ms, dt, lo, hi = "burgers", 2, (4, 3), [8, 4], [5, 3], 5e-3, [0, 0], [1, 1]
    else:
        eq, dim, n, Ps, Ms, dt, lo, hi = "ns", 3, (2, 3, 2), [4, 2], [3, 2], 4e-3, [0] * 3, [2 * np.pi] * 3
    prob = lib_problem(S, eq, dim, n, lo, hi, nu=5e-3 if eq == "burgers" else 0.01)
    prec = S.MIXED if precision == "mixed" else S.FP64
    meth = S.make_method(Ps, Ms, n_iter=3 if len(Ps) == 1 else 2, cg_rtol=1e-12, cg_maxit=4000, precision=prec)
    sv = S.Solver(prob, meth)
    phys = oracle_phys(eq, dim, nu=5e-3 if eq == "burgers" else 0.01)
    levels = [DGLevel(phys, n, lo, hi, P, M, rtol=1e-14) for P, M in zip(Ps, Ms)]
    fine = levels[0]
    if eq == "ns":
        from paper_2504_18526_amd.inputs import taylor_green
        u = taylor_green(fine.coords(), mach=0.1)
    else:
        u = smooth_state(phys, fine, np.random.default_rng(4))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for lvl in range(len(Ps)):
        sv.net_init(lvl, 32, seed=2 + lvl, max_batch=512, max_rows=20000)
        sv.net_harvest(lvl, 1)
    sv.set_state(dev(u.ravel()))
    for _ in range(2):
        sv.step(dt)
    for lvl in range(len(Ps)):
        sv.net_harvest(lvl, 0)
        sv.net_train(lvl, 30, 256, 1e-3)
        sv.net_use(lvl, 1)
    if len(Ps) == 1:
        stepper = lambda v: sdc_step(fine, v, dt, 3)
    else:
        ml = MLSDC(list(reversed(levels)), n_coarse=2, start="cascade", cycles=2, post_sweep=True)
        stepper = lambda v: ml.step(v, dt)
    state = torch.empty(u.size, dtype=torch.float64, device="cuda")
    sv.get_state(state)
    cur = state.cpu().numpy().reshape(u.shape)
    guesses = 0
    for k in range(3):
        sv.set_state(dev(cur.ravel()))
        st = sv.step(dt)
        guesses += st["net_guesses"]
        sv.get_state(state)
        got = state.cpu().numpy().reshape(u.shape)
        ref = stepper(cur)
        assert rel_l2(got, ref) < 1e-10, (case, precision, k)
        assert st["not_converged"] == 0
        cur = got
    assert guesses > 0
    sv.close()
