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
