"""Workload definitions (sizes, time steps, initial data) shaped like the
paper's test problems, as C-ABI problem / method descriptors.

Time steps follow the paper's CFL definition (Sec. 8, eq. cfl):
CFL = dt lam_c,max / dx, dx = dx_e / (2 delta(P)), where delta(P) is taken
as the largest |eigenvalue| of the GLL collocation derivative matrix on
[-1, 1] with the inflow node removed (reading of the paper's "largest
eigenvalue of the convection problem with one-sided Dirichlet conditions";
the table is verified by a CPU test).  In d dimensions lam_c,max is the sum
over d of the largest directional wave speed.
"""
DELTA = {2: 1.000, 3: 1.665, 4: 2.472, 5: 3.409, 6: 4.471, 7: 5.656, 8: 6.967}


def cfl_dt(cfl, h, P, lam):
    return cfl * (h / (2.0 * DELTA[P])) / lam


def burgers_2level():
    """Two-level SI-MLSDC for 2-D viscous Burgers on [0,1]^2: 32 x 32
    elements, fine P = 8 / M = 5, coarse P = 4 / M = 3, nu = 5e-3, cascade
    start, 3 V-cycles + fine post-sweep, N_c = 2, CFL = 2 (lam = 2 max|u0|
    = 2), 200 steps, u0 from seeded Fourier modes |k| <= 6, amplitude
    1/|k|^2, scaled to max |u0| = 1."""
    return dict(
        name="burgers2d_mlsdc_32x32_P8-4_M5-3",
        eq="burgers", dim=2, n_elem=(32, 32), lo=(0.0, 0.0), hi=(1.0, 1.0), nu=5e-3,
        P=[8, 4], M=[5, 3], start="cascade", cycles=3, n_coarse=2, post_sweep=1,
        dt=cfl_dt(2.0, 1.0 / 32, 8, 2.0), steps=200, seed=0, kmax=6,
        cg_rtol=1e-10,
    )


def convdiff_1level():
    """Single-level SI-SDC for 2-D convection-diffusion on [0,1]^2:
    a = (1, 0.5), nu = 0.01, 8 x 8 elements, P = 4, M = 3, 4 sweeps, CFL = 1
    (lam = |a_x| + |a_y| = 1.5), 100 steps, u0 = sin 2pi x sin 2pi y + seeded
    Fourier modes |k| <= 4 with N(0,1)/|k|^2 amplitudes."""
    return dict(
        name="convdiff2d_sdc_8x8_P4_M3",
        eq="convdiff", dim=2, n_elem=(8, 8), lo=(0.0, 0.0), hi=(1.0, 1.0), nu=0.01, a=(1.0, 0.5),
        P=[4], M=[3], start="cascade", cycles=4, n_coarse=2, post_sweep=0,
        dt=cfl_dt(1.0, 1.0 / 8, 4, 1.5), steps=100, seed=0, kmax=4,
        cg_rtol=1e-10,
    )


def fine_sweeps_per_step(w):
    """Predictor + corrector sweeps on the finest level per step: one
    level: predictor + K sweeps; cascade / FMG starts do no fine sweep, then
    C V-cycles (one fine pre-sweep each) and the optional post-sweep."""
    if len(w["P"]) == 1:
        return 1 + w["cycles"]
    return w["cycles"] + (1 if w["post_sweep"] else 0)


def euler_3level():
    """Three-level SI-MLSDC, 2-D Euler isentropic vortex on [0,10]^2 (eps = 5,
    background Mach 0.5 along +x, gamma = 1.4): 64 x 64 elements, P 6/4/2,
    M 5/3/2, FMG start, 3 V-cycles + post-sweep, N_c = 2, CFL = 4 with lam =
    max over nodes of sum_d (|v_d| + c) of u0, 40 steps."""
    return dict(
        name="euler2d_vortex_mlsdc_64x64_P6-4-2_M5-3-2",
        eq="euler", dim=2, n_elem=(64, 64), lo=(0.0, 0.0), hi=(10.0, 10.0), gamma=1.4,
        P=[6, 4, 2], M=[5, 3, 2], start="fmg", cycles=3, n_coarse=2, post_sweep=1,
        cfl=4.0, steps=40, cg_rtol=1e-10,
    )


def ns_2level():
    """Two-level SI-MLSDC, 3-D compressible Navier-Stokes Taylor-Green
    vortex on [0, 2 pi]^3: 16^3 hexahedra, P 7/3, M 4/2, Re = 1600 (mu =
    1/1600 with rho0 = V0 = L = 1), Ma = 0.1, Pr = 0.71, gamma = 1.4, R = 1;
    cascade start, 3 V-cycles + post-sweep, N_c = 2, CFL = 8 with the
    acoustic lam = max sum_d (|v_d| + c), 10 steps."""
    return dict(
        name="ns3d_taylor_green_mlsdc_16^3_P7-3_M4-2",
        eq="ns", dim=3, n_elem=(16, 16, 16), lo=(0.0, 0.0, 0.0), hi=(6.283185307179586,) * 3,
        gamma=1.4, mu=1.0 / 1600.0, Pr=0.71, mach=0.1,
        P=[7, 3], M=[4, 2], start="cascade", cycles=3, n_coarse=2, post_sweep=1,
        cfl=8.0, steps=10, cg_rtol=1e-10,
    )


def systems_dt(w, u0):
    """dt from the CFL number for the Euler / Navier-Stokes workloads:
    lam = max over nodes of sum_d (|v_d| + c) of the initial state u0
    (conservative variables [var][...])."""
    import numpy as np
    g = w["gamma"]
    dim = w["dim"]
    rho = u0[0]
    v = [u0[1 + d] / rho for d in range(dim)]
    p = (g - 1.0) * (u0[dim + 1] - 0.5 * rho * sum(vd * vd for vd in v))
    c = np.sqrt(g * p / rho)
    lam = float(np.max(sum(np.abs(vd) + c for vd in v)))
    h = (w["hi"][0] - w["lo"][0]) / w["n_elem"][0]
    return cfl_dt(w["cfl"], h, w["P"][0], lam)


def batch_instances(n=64, base_seed=0):
    """Batched serving-shape run: n independent 2-D instances on [0,1]^2,
    instance i drawn with numpy.random.default_rng(base_seed + i):
    elements m x m with m = round(exp U[ln 8, ln 64]); P uniform in 3..8;
    M uniform in {3, 4, 5}; nu log-uniform in [1e-3, 1e-1]; even i
    convection-diffusion (a = (1, 0.5), u0 as in the one-level workload),
    odd i Burgers (u0 as in the two-level workload); two levels with
    P_c = ceil(P/2), M_c = floor(M/2) + 1 (the paper's coarsening rule);
    cascade start, 3 V-cycles + post-sweep, N_c = 2, CFL = 1, 20 steps,
    mixed precision with FP64 refinement, PCG to 1e-10."""
    import math
    import numpy as np
    out = []
    for i in range(n):
        rng = np.random.default_rng(base_seed + i)
        m = int(round(math.exp(rng.uniform(math.log(8.0), math.log(64.0)))))
        P = int(rng.integers(3, 9))
        M = int(rng.integers(3, 6))
        nu = float(math.exp(rng.uniform(math.log(1e-3), math.log(1e-1))))
        eq = "convdiff" if i % 2 == 0 else "burgers"
        lam = 1.5 if eq == "convdiff" else 2.0
        out.append(dict(
            name=f"instance{i}", eq=eq, dim=2, n_elem=(m, m), lo=(0.0, 0.0), hi=(1.0, 1.0), nu=nu,
            a=(1.0, 0.5, 0.0), P=[P, (P + 1) // 2], M=[M, M // 2 + 1], start="cascade", cycles=3, n_coarse=2,
            post_sweep=1, dt=cfl_dt(1.0, 1.0 / m, P, lam), steps=20, seed=base_seed + i,
            kmax=4 if eq == "convdiff" else 6, cg_rtol=1e-10, precision="mixed",
        ))
    return out


def batch_64():
    """The 64-instance batch as one workload record (instances in `instances`)."""
    inst = batch_instances(64)
    return dict(name="batch2d_64_instances_mlsdc_mixed", eq="batch", dim=2, instances=inst, steps=20)


def burgers_ensemble():
    """Ensemble: 64 independent instances of the two-level Burgers
    configuration (P 8/4, M 5/3, nu = 5e-3, cascade, 3 V-cycles + post-sweep,
    N_c = 2) on 16 x 16-element boxes [0,1]^2, instance k with u0 from
    seeded Fourier modes (seed k, |k| <= 6, scaled to max |u0| = 1), one
    shared dt (CFL 2 on h = 1/16), 20 steps; stacked in one handle (problem
    `stack`), no conservation shift."""
    return dict(
        name="burgers2d_ensemble_64x16x16_P8-4_M5-3",
        eq="burgers", dim=2, n_elem=(16, 16), lo=(0.0, 0.0), hi=(1.0, 1.0), nu=5e-3,
        P=[8, 4], M=[5, 3], start="cascade", cycles=3, n_coarse=2, post_sweep=1,
        dt=cfl_dt(2.0, 1.0 / 16, 8, 2.0), steps=20, seed=0, kmax=6, cg_rtol=1e-10,
        stack=64, conserve=0,
    )


def sod_2level():
    """Shock workload shaped like the paper's Sod test (Sec. 8: 80 elements of
    degree 5 on [0, 1], levels P 5/3, M 7/5, 32 steps to t = 0.2, cascade
    start, artificial viscosity kappa_s = 2, c_s = 0.4): 2-D Euler on the
    periodic strip [0, 2] x [0, 1/80] with a pair of Sod tubes
    (inputs.sod_pair, jumps smoothed over 0.2 h), 160 x 1 elements of size
    1/80, 2 V-cycles + post-sweep, N_c = 2."""
    return dict(
        name="euler2d_sod_pair_av_160x1_P5-3_M7-5",
        eq="euler", dim=2, n_elem=(160, 1), lo=(0.0, 0.0), hi=(2.0, 1.0 / 80), gamma=1.4,
        P=[5, 3], M=[7, 5], start="cascade", cycles=2, n_coarse=2, post_sweep=1,
        dt=0.2 / 32, steps=32, cg_rtol=1e-10, av=(2.0, 0.4), init="sod",
    )


WORKLOADS = {
    "convdiff": convdiff_1level,
    "burgers": burgers_2level,
    "euler": euler_3level,
    "ns": ns_2level,
    "batch": batch_64,
    "sod": sod_2level,
    "ensemble": burgers_ensemble,
}
