"""Pin of the oracle's finite-cycle MLSDC (Alg. 2 V-cycle, Alg. 3 cascade
start) on the scalar test equation of Sec. 5, against the same steps written
out by hand for the smallest two-level case.

Levels: fine M_f = 2 Radau-right nodes tau = (1/3, 1), coarse M_c = 1 node
tau = (1); dt = 1, u_0 = 1.  Tables, derived by hand:
  * fine node-to-node weights (eq. nn_weights): the Radau IIA matrix of M = 2
    is [[5/12, -1/12], [3/4, 1/4]]; its first row and the difference of its
    rows give w^nn = [[5/12, -1/12], [1/3, 1/3]];  coarse w^nn = [[1]];
  * I_t (fine x coarse) = [[1], [1]] (the one coarse Lagrange polynomial is
    the constant 1); P_t (coarse x fine) = [0, 1] (tau_c = 1 is the fine node
    2); R_t = I_t^T = [1, 1] (eq. restriction).
Scalar operators (eq. dahlquist): mass 1, C(u) = i lam_i u, f(u) = z u,
implicit coefficient K_m = (dt_m/2) lam_i^2 - lam_r (eq. H_SI(1)), solve
x = b / (1 + dt_m K_m).  g enters both SI(2) stages (the reading that keeps
the collocation solution a fixed point).

The hand version fixes the number of coarse sweeps N_c = 2, the order
pre-sweep -> residual -> projection -> FAS right-hand side -> coarse sweeps ->
correction prolongation -> post-sweep, and the signs r = g - F(u),
g_c = F_c(P u) + R r, u += I (u_c - v); a change of any of them in the
oracle moves R(z) at the 1e-2 level for these z.  CPU only.
"""
import numpy as np
import pytest

from oracle import dahlquist

WF = np.array([[5.0 / 12.0, -1.0 / 12.0], [1.0 / 3.0, 1.0 / 3.0]])
DTF = np.array([1.0 / 3.0, 2.0 / 3.0])


def _sweep(z, U, g, w, dts, scheme):
    """One SI(1)/SI(2) corrector sweep on nodes 1..M of U (U[0] = u_0)."""
    li, lr = z.imag, z.real
    M = len(dts)
    q = [None] + [sum(w[m, i] * z * U[i + 1] for i in range(M)) for m in range(M)]
    new = [U[0]]
    for m in range(1, M + 1):
        d = dts[m - 1]
        K = 0.5 * d * li * li - lr
        gm = g[m] if g is not None else 0.0
        h1_old = d * (1j * li * U[m - 1] - K * U[m])
        y = (new[m - 1] + q[m] + gm + d * 1j * li * new[m - 1] - h1_old) / (1 + d * K)
        if scheme == "si1":
            new.append(y)
            continue
        h2_old = d * (1j * li * U[m] - K * U[m])
        new.append((new[m - 1] + q[m] + gm + d * 1j * li * y - h2_old) / (1 + d * K))
    return new


def _residual(z, U, w):
    """F_m(U) = (U_m - U_{m-1}) - q_m(U)."""
    M = w.shape[0]
    return [None] + [(U[m] - U[m - 1]) - sum(w[m - 1, i] * z * U[i + 1] for i in range(M))
                     for m in range(1, M + 1)]


def hand_two_level(z, scheme, cycles, post, n_coarse=2):
    li, lr = z.imag, z.real
    u0 = 1.0 + 0.0j
    Kc = 0.5 * li * li - lr
    # Alg. 3: coarse predictor, one coarse sweep (g = 0), interpolation
    y = (u0 + 1j * li * u0) / (1 + Kc)
    uc1 = y if scheme == "si1" else (u0 + 1j * li * y) / (1 + Kc)
    Uc = _sweep(z, [u0, uc1], None, np.array([[1.0]]), [1.0], scheme)
    Uf = [u0, Uc[1], Uc[1]]                    # I_t = [[1], [1]]
    for _ in range(cycles):                    # Alg. 2
        Uf = _sweep(z, Uf, None, WF, DTF, scheme)          # pre-sweep, g_f = 0
        Ff = _residual(z, Uf, WF)
        r = [None, -Ff[1], -Ff[2]]                         # r = 0 - F_f(u_f)
        v = [u0, Uf[2]]                                    # P_t = [0, 1]
        Fc = _residual(z, v, np.array([[1.0]]))
        gc = [None, Fc[1] + r[1] + r[2]]                   # R_t = [1, 1]
        Uc = list(v)
        for _ in range(n_coarse):
            Uc = _sweep(z, Uc, gc, np.array([[1.0]]), [1.0], scheme)
        corr = Uc[1] - v[1]
        Uf = [u0, Uf[1] + corr, Uf[2] + corr]              # I_t (u_c - v)
    if post:
        Uf = _sweep(z, Uf, None, WF, DTF, scheme)
    return Uf[2]


ZS = [-0.5 + 0.3j, -2.0 + 1.5j, -0.2 - 1.1j]


@pytest.mark.parametrize("scheme", ["si1", "si2"])
@pytest.mark.parametrize("cycles,post", [(1, True), (1, False), (3, True)])
def test_two_level_vcycle_matches_hand_steps(scheme, cycles, post):
    for z in ZS:
        want = hand_two_level(z, scheme, cycles, post)
        got = dahlquist.amplification_mlsdc(z, [1, 2], cycles, scheme=scheme, n_coarse=2,
                                            start="cascade", post_sweep=post)
        assert abs(got - want) < 1e-14 * max(1.0, abs(want)), (z, got, want)


def test_hand_steps_are_sensitive_to_the_pinned_choices():
    """The pinned choices matter at these z: N_c = 1 or a reversed FAS sign
    gives a different R(z) (so the pin above can tell them apart)."""
    z = ZS[1]
    base = hand_two_level(z, "si2", 1, True)
    assert abs(hand_two_level(z, "si2", 1, True, n_coarse=1) - base) > 1e-3
    assert abs(hand_two_level(z, "si2", 1, True, n_coarse=3) - base) > 1e-4


def test_hand_steps_converge_to_radau_iia_m2():
    """Sanity of the hand version itself: many cycles reach the fine
    collocation solution, the (1, 2) Pade approximant of e^z (Radau IIA, M = 2)."""
    for z in ZS:
        R = hand_two_level(z, "si2", 60, True)
        pade = (1 + z / 3) / (1 - 2 * z / 3 + z * z / 6)
        assert abs(R - pade) < 1e-12


def pade(z, m, n):
    """(m, n) Pade approximant of e^z (closed form)."""
    from math import factorial
    N = sum(factorial(m + n - j) * factorial(m) / (factorial(m + n) * factorial(j) * factorial(m - j)) * z ** j
            for j in range(m + 1))
    D = sum(factorial(m + n - j) * factorial(n) / (factorial(m + n) * factorial(j) * factorial(n - j)) * (-z) ** j
            for j in range(n + 1))
    return N / D


@pytest.mark.parametrize("z", ZS[:2])
def test_fmg_start_with_many_cycles_solves_the_middle_level(z):
    """Alg. 4 with C_fmg V-cycles on the two coarsest levels of three: as
    C_fmg grows, the middle level reaches its own collocation solution (a
    two-level V-cycle with g = 0 on its top level has it as fixed point): at
    its last node the (M-1, M) Pade approximant of e^z for M = 3 Radau nodes.
    One cycle per level is not yet there, so the pin sees C_fmg."""
    ml = dahlquist.mlsdc(z.real, z.imag, [2, 3, 5], start="fmg", cycles=0, post_sweep=False, c_fmg=40,
                         scheme="si2", n_coarse=2)
    ml.set_initial(np.complex128(1.0), None)
    ml.start_levels(1.0)
    assert abs(ml.U[1][-1] - pade(z, 2, 3)) < 1e-12
    one = dahlquist.mlsdc(z.real, z.imag, [2, 3, 5], start="fmg", cycles=0, post_sweep=False, c_fmg=1,
                          scheme="si2", n_coarse=2)
    one.set_initial(np.complex128(1.0), None)
    one.start_levels(1.0)
    assert abs(one.U[1][-1] - pade(z, 2, 3)) > 1e-6   # one cycle per level is not yet converged


def test_constant_start_spreads_u0_and_converges():
    """The constant start puts u_0 on every node of every level; V-cycles from
    it converge to the fine collocation solution (Radau IIA, the (M-1, M) Pade
    approximant), and it needs at least as many cycles as the predictor start
    for a given accuracy (Sec. 7, test 4 observes one more)."""
    z = -1.0 + 0.8j
    ml = dahlquist.mlsdc(z.real, z.imag, [2, 3], start="constant", cycles=0, post_sweep=False)
    ml.set_initial(np.complex128(1.0), None)
    ml.start_levels(1.0)
    for i in range(2):
        assert all(u == 1.0 for u in ml.U[i])
    assert abs(dahlquist.amplification_mlsdc(z, [2, 3], 40, start="constant") - pade(z, 2, 3)) < 1e-12
    errs = {}
    for start in ("constant", "predictor"):
        errs[start] = [abs(dahlquist.amplification_mlsdc(z, [2, 3], c, start=start) - pade(z, 2, 3))
                       for c in range(1, 6)]
    assert sum(errs["constant"]) > sum(errs["predictor"])
