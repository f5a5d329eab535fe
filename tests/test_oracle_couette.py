"""Whole-scheme pins of the Couette oracle (arXiv:1708.05944, Secs. III and V).

Each pin is fixed by the paper's analysis or by mathematics, not by the oracle itself:
exact particle-number conservation (Sec. III.D), stationarity of the rest state
(Sec. V.C.2, Eq. f_st), third-order time stepping (Sec. III.A), the rigid-rotation
solution (Sec. V.C.3, Eqs. rigid_sol and rigid_density), the Navier-Stokes Couette
velocity and temperature profiles (Sec. V.D, Eqs. NS_U and NS_T), the steady-state
invariants of Sec. V.B (Eqs. TRph and Q_def, and u^R = 0), and the Butcher tableau of
Table rk3 (tests/golden/rk3_butcher.txt) against the oracle's time step.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.couette import TAU_AOKI, TAU_HYDRO, CouetteOracle


def _perturbed(o, seed):
    """A positive, non-equilibrium state: local equilibria with varying (n, u, T) times
    random per-velocity factors."""
    rng = np.random.default_rng(seed)
    R = o.Rc
    F = o.equilibrium(1 + 0.1 * np.sin(3 * R), 0.05 * np.cos(2 * R), 0.2 * np.sin(R), 1 + 0.1 * np.cos(R))
    return F * rng.uniform(0.8, 1.2, F.shape)


REST_CASES = [
    dict(ax1=(0, 5, 4), ax2=(0, 5, 4), Kn=1e-3, tau_model=TAU_HYDRO, A=0.0),
    dict(ax1=(0, 5, 4), ax2=(0, 5, 4), Kn=1e-3, tau_model=TAU_HYDRO, A=0.95),
    dict(ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1, tau_model=TAU_AOKI, A=0.95),
    dict(ax1=(1, 8, 4), ax2=(1, 4, 3), Kn=1.0, tau_model=TAU_AOKI, A=0.0),
]


@pytest.mark.parametrize("case", REST_CASES)
def test_rest_state_is_stationary(case):
    """Both cylinders at rest: f' = f'_eq(1, 0, 1), f'' = f' solves the discrete scheme to
    rounding (advection cancelled by the force term, walls at n_w = 1), with and
    without grid stretching."""
    o = CouetteOracle(N_R=16, u_in=0.0, **case)
    F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    L, nw = o.L(F)
    tau = case["Kn"] if case["tau_model"] == TAU_HYDRO else case["Kn"] * math.sqrt(math.pi / 8)
    assert np.abs(L).max() <= 1e-13 * max(1.0, 1.0 / tau)
    assert np.allclose(nw, 1.0, atol=1e-14)
    F2 = o.step(F, o.cfl_dt(0.5) if case["Kn"] > 0.01 else 1e-3, 100)
    assert np.abs(F2 - F).max() <= 1e-13


MASS_CASES = [
    dict(ax1=(1, 4, 2), ax2=(0, 4, 2), A=0.0),
    dict(ax1=(1, 4, 2), ax2=(0, 4, 2), A=0.95),
    dict(ax1=(0, 5, 4), ax2=(0, 5, 4), A=0.5),
    dict(ax1=(1, 6, 4), ax2=(1, 3, 2), A=0.0),
]


@pytest.mark.parametrize("case", MASS_CASES)
def test_operator_conserves_particle_number(case):
    """sum_s dchi_s sum_k L'[F]_{s,k} = 0 for an arbitrary state (Sec. III.D): the bulk
    fluxes telescope, the wall fluxes vanish by Eq. nw, and the force and collision
    terms have zero zeroth moment."""
    o = CouetteOracle(N_R=12, u_in=0.3, u_out=-0.1, T_out=1.2, **case)
    F = _perturbed(o, 7)
    L, _ = o.L(F)
    dN = (o.dchi[:, None] * L[0]).sum()
    scale = (o.dchi[:, None] * np.abs(L[0])).sum()
    assert abs(dN) <= 1e-14 * scale


def test_particle_number_constant_over_many_steps():
    """N_tot drifts by rounding only over 10^4 RK3 steps with a rotating inner wall:
    the bound is 10^4 steps times one unit roundoff (2.2e-16) per step."""
    o = CouetteOracle(N_R=32, u_in=0.1)
    F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    m0 = o.mass(F)
    F = o.step(F, o.cfl_dt(0.5), 10000)
    assert abs(o.mass(F) / m0 - 1) <= 1e4 * 2.2e-16


def test_rk3_is_third_order_in_time():
    """At a fixed grid, the error of Eq. rk3 at a fixed final time falls ~8x per halving
    of dt (Table rk3 is the third-order Shu-Osher scheme)."""
    o = CouetteOracle(N_R=16, u_in=0.3)
    F0 = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    dt0 = o.cfl_dt(0.5)
    ref = o.step(F0, dt0 / 16, 40 * 16)
    e = [np.abs(o.step(F0, dt0 / k, 40 * k) - ref).max() for k in (2, 4)]
    assert 6.0 < e[0] / e[1] < 10.5, e


def _butcher(path=os.path.join(os.path.dirname(__file__), "golden", "rk3_butcher.txt")):
    """(c, A, b) of tests/golden/rk3_butcher.txt (Table rk3), as exact fractions."""
    rows = [ln.split("|") for ln in open(path) if ln.strip() and not ln.startswith("#")]
    c, A, b = [], [], None
    for left, right in rows:
        vals = [Fraction(x) for x in right.split()]
        if left.strip() == "b":
            b = vals
        else:
            c.append(Fraction(left.strip()))
            A.append(vals)
    return c, A, b


def test_rk3_butcher_tableau_golden():
    """One oracle RK3 step equals the Runge-Kutta step built from the golden Butcher
    tableau of Table rk3 (stages k_i = L[F + dt sum_j a_ij k_j], F + dt sum b_i k_i) with the
    oracle's operator L, to rounding; the tableau itself is consistent (rows of A sum to c,
    b sums to 1, third-order conditions) and a perturbed weight is detected."""
    c, A, b = _butcher()
    assert [sum(r) for r in A] == c and sum(b) == 1
    assert sum(bi * ci for bi, ci in zip(b, c)) == Fraction(1, 2)
    assert sum(bi * ci * ci for bi, ci in zip(b, c)) == Fraction(1, 3)
    assert sum(b[i] * A[i][j] * c[j] for i in range(3) for j in range(3)) == Fraction(1, 6)
    o = CouetteOracle(N_R=12, u_in=0.3, T_in=1.1)
    rng = np.random.default_rng(5)
    F = o.equilibrium(1.0, 0.0, 0.05, 1.0) * (1 + 0.05 * rng.standard_normal((2, 12, o.NV)))
    dt = o.cfl_dt(0.5)

    def tableau_step(bw):
        ks = []
        for i in range(3):
            Fi = F + dt * sum(float(A[i][j]) * ks[j] for j in range(i)) if i else F
            ks.append(o.L(Fi)[0])
        return F + dt * sum(float(bi) * k for bi, k in zip(bw, ks))

    got = o.step(F, dt, 1)
    want = tableau_step(b)
    scale = np.abs(want - F).max()
    assert np.abs(got - want).max() <= 1e-12 * scale + 1e-15 * np.abs(F).max()
    wrong = tableau_step([b[0], b[1] + Fraction(1, 100), b[2] - Fraction(1, 100)])
    assert np.abs(got - wrong).max() > 1e-6 * scale


def _run_to(o, F, dt, tol, chunk=500, max_steps=100000):
    steps = 0
    r = math.inf
    while steps < max_steps:
        F = o.step(F, dt, chunk)
        Fn = o.step(F, dt, 1)
        steps += chunk + 1
        r = o.residual(Fn, F, dt)
        F = Fn
        if r < tol:
            break
    return F, steps, r


def _n_rigid(R, Om, Rin, Rout):
    """Eq. rigid_density with m = T_w = 1 and N_tot = pi (R_out^2 - R_in^2)."""
    c = Om ** 2 / 4
    Ntot = math.pi * (Rout ** 2 - Rin ** 2)
    return Ntot * Om ** 2 / (4 * math.pi) * np.exp(c * (2 * R ** 2 - Rin ** 2 - Rout ** 2)) / math.sinh(
        c * (Rout ** 2 - Rin ** 2))


@pytest.mark.slow
def test_rigid_rotation_converges_to_analytic_solution():
    """Both cylinders at the same angular speed: the steady state approaches
    f_eq(n(R), Omega R, T_w) (Eqs. rigid_sol, rigid_density) as the grid is refined; the
    residual deviation comes from the wall ghost layer and shrinks with delta R."""
    Om, Rin, Rout = 0.1, 1.0, 2.0
    devs = []
    for NR in (16, 32):
        o = CouetteOracle(N_R=NR, ax1=(0, 5, 4), ax2=(0, 5, 4), Kn=0.1, tau_model=TAU_AOKI,
                          u_in=Om * Rin, u_out=Om * Rout)
        F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
        F, steps, r = _run_to(o, F, o.cfl_dt(0.5), 1e-9)
        assert r < 1e-9
        m = o.moments(F)
        R = o.Rc
        du = np.abs(m["u2"] - Om * R).max() / (Om * Rout)
        dn = np.abs(m["n"] - _n_rigid(R, Om, Rin, Rout)).max()
        devs.append(max(du, dn))
    assert devs[1] < 0.75 * devs[0], devs
    assert devs[1] < 5e-3, devs


@pytest.mark.slow
def test_navier_stokes_couette_profile():
    """Near the hydrodynamic limit (tau = Kn/(nT), Eq. hydro_tau) the steady u^phi
    approaches Eq. NS_U, u = A R + B/R with A = -1/30, B = 2/15 for Omega_in = 0.1,
    R_in = 1, R_out = 2; the deviation is the velocity slip, first order in Kn."""
    Om, Rin, Rout = 0.1, 1.0, 2.0
    B = Om / (Rin ** -2 - Rout ** -2)
    A = -Om * Rin ** 2 / (Rout ** 2 - Rin ** 2)
    assert abs(A + 1 / 30) < 1e-15 and abs(B - 2 / 15) < 1e-15
    errs = []
    for Kn in (0.01, 0.005):
        o = CouetteOracle(N_R=32, ax1=(0, 5, 4), ax2=(0, 5, 4), Kn=Kn, tau_model=TAU_HYDRO, u_in=Om * Rin)
        R = o.Rc
        u_ns = A * R + B / R
        F = o.equilibrium(1.0, 0.0, u_ns, 1.0)
        F, steps, r = _run_to(o, F, min(o.cfl_dt(0.5), 2 * Kn), 1e-7)
        m = o.moments(F)
        errs.append(np.abs(m["u2"] - u_ns).max() / (Om * Rin))
    assert errs[0] < 5 * 0.01 and errs[1] < 5 * 0.005, errs
    assert 1.6 < errs[0] / errs[1] < 2.6, errs


def _ns_limit_runs(Om, Kns, NR=32, tol=1e-8):
    """Steady states near the hydrodynamic limit (tau = Kn/(nT), Eq. hydro_tau, so mu = Kn
    and kappa = 5 mu / 2 are constant, as Eqs. NS_U and NS_T assume), started from the
    Navier-Stokes profiles; returns (R, [moments per Kn])."""
    Rin, Rout = 1.0, 2.0
    a = Rin ** -2 - Rout ** -2
    out = []
    for Kn in Kns:
        o = CouetteOracle(N_R=NR, ax1=(0, 5, 4), ax2=(0, 5, 4), Kn=Kn, tau_model=TAU_HYDRO, u_in=Om * Rin)
        R = o.Rc
        F = o.equilibrium(1.0, 0.0, _u_ns(R, Om), _T_ns(R, Om))
        F, steps, r = _run_to(o, F, min(o.cfl_dt(0.5), 2 * Kn), tol, chunk=999)
        assert r < tol
        out.append(o.moments(F))
    return R, out


def _u_ns(R, Om, Rin=1.0, Rout=2.0):
    """Eq. NS_U."""
    return R ** -1 * Om / (Rin ** -2 - Rout ** -2) - R * Om * Rin ** 2 / (Rout ** 2 - Rin ** 2)


def _T_ns(R, Om, Rin=1.0, Rout=2.0, Tw=1.0, mu_over_kappa=0.4):
    """Eq. NS_T, with mu / kappa = 2/5 (BGK: Prandtl number 1, c_p = 5/2 for m = 1)."""
    a = Rin ** -2 - Rout ** -2
    return Tw + mu_over_kappa * Om ** 2 / a * ((Rin ** -2 - R ** -2) / a - np.log(R / Rin) / np.log(Rout / Rin))


@pytest.mark.slow
def test_navier_stokes_temperature_profile():
    """At Omega_in = 0.5 the viscous heating lifts T by ~2 % in the gap; near the
    hydrodynamic limit the steady T - T_w approaches Eq. NS_T (constant mu and kappa =
    5 mu/2), the deviation being the temperature jump and velocity slip at the walls,
    first order in Kn (measured: 13 Kn of the peak rise at Kn = 0.01 and 0.005).  A dropped
    energy term (the f'' channel, the heat flux, the viscous heating) would miss the rise
    entirely.  Richardson extrapolation in Kn (2 X(Kn/2) - X(Kn)) removes the first-order
    part: the extrapolated u^phi is within 1e-2 Omega_in R_in of Eq. NS_U (measured 8.7e-3:
    the O(Kn^2) slip and the 32-cell discretisation) and the extrapolated T rise within 2 %
    of Eq. NS_T's (measured 1.5 %)."""
    Om = 0.5
    R, (m1, m2) = _ns_limit_runs(Om, (0.01, 0.005))
    dTn = _T_ns(R, Om) - 1.0
    eT = [np.abs((m["T"] - 1.0) - dTn).max() / dTn.max() for m in (m1, m2)]
    assert abs(dTn.max() - 0.0225) < 5e-4
    assert eT[0] < 20 * 0.01 and eT[1] < 20 * 0.005, eT
    assert 1.6 < eT[0] / eT[1] < 2.6, eT
    u_x = 2 * m2["u2"] - m1["u2"]
    T_x = 2 * m2["T"] - m1["T"]
    eu_x = np.abs(u_x - _u_ns(R, Om)).max() / Om
    eT_x = np.abs((T_x - 1.0) - dTn).max() / dTn.max()
    assert eu_x < 1e-2, eu_x
    assert eT_x < 2e-2, eT_x


@pytest.mark.slow
def test_transition_regime_steady_invariants():
    """Workload of the single-instance benchmark (R = 1..2, u_w = 0.1, Kn = 0.1,
    HH(2;4) x H(2;4), 64 cells): at steady state u^R -> 0, R^2 T^{R phi} and
    R (q^R + u^phi T^{R phi}) are constant up to discretisation error (Sec. V.B),
    and the error shrinks when the grid is refined."""
    spreads = []
    for NR in (32, 64):
        o = CouetteOracle(N_R=NR)
        F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
        F, steps, r = _run_to(o, F, o.cfl_dt(0.5), 1e-10)
        assert r < 1e-10
        m = o.moments(F)
        R = o.Rc
        assert np.abs(m["u1"]).max() < 1e-5
        tr = R ** 2 * m["T12"]
        qq = R * (m["q1"] + m["u2"] * m["T12"])
        spreads.append((np.ptp(tr) / abs(tr.mean()), np.ptp(qq) / abs(qq.mean())))
    assert spreads[1][0] < 0.6 * spreads[0][0] and spreads[1][0] < 0.02, spreads
    assert spreads[1][1] < 0.6 * spreads[0][1] and spreads[1][1] < 0.02, spreads
