"""Pins of the optional regularised WENO-5 weights (an extension: weno_eps = 0 is the
paper's epsilon-free scheme of Sec. III.C, Table weno)."""
import numpy as np
import pytest

from oracle.couette import CouetteOracle, weno5, weno5_eps


def _data(seed, n=200):
    return np.random.default_rng(seed).normal(size=(n, 5))


def test_zero_eps_is_the_epsilon_free_scheme():
    for a, b, c, d, e in _data(1):
        assert weno5_eps(a, b, c, d, e, 0.0) == weno5(a, b, c, d, e)


def test_large_eps_gives_the_linear_fifth_order_scheme():
    """Ideal weights (0.1, 0.6, 0.3) combine the three candidate parabolas into the
    upwind-biased linear 5th-order interpolant (2a - 13b + 47c + 27d - 3e)/60."""
    for a, b, c, d, e in _data(2):
        lin = (2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60
        assert weno5_eps(a, b, c, d, e, 1e30) == pytest.approx(lin, rel=1e-12, abs=1e-13)


def test_regularised_flux_is_homogeneous_of_degree_one():
    for a, b, c, d, e in _data(3, 50):
        for lam in (1e-12, 3.7, 1e9):
            assert weno5_eps(lam * a, lam * b, lam * c, lam * d, lam * e, 1e-6) == pytest.approx(
                lam * weno5_eps(a, b, c, d, e, 1e-6), rel=1e-13)


def test_exactly_vanishing_indicator_keeps_the_table_limit():
    """A constant upwind stencil (the all-ghost wall stencil) keeps the weights of
    Table weno whatever eps, so the emitted wall flux stays the ghost Maxwellian (to the
    rounding of the candidate parabola)."""
    for g, d, e in np.random.default_rng(4).normal(size=(50, 3)):
        for eps in (1e-6, 1.0):
            assert weno5_eps(g, g, g, d, e, eps) == weno5(g, g, g, d, e)
        assert weno5_eps(g, g, g, d, e, 1.0) == pytest.approx(g, rel=1e-15, abs=1e-300)


def test_regularisation_moves_weights_toward_ideal_continuously():
    """Between the limits the flux varies continuously with eps (monotone approach of
    the linear scheme on a steep stencil)."""
    a, b, c, d, e = 0.0, 0.0, 1.0, 10.0, 10.5
    lin = (2 * a - 13 * b + 47 * c + 27 * d - 3 * e) / 60
    vals = [weno5_eps(a, b, c, d, e, eps) for eps in (0.0, 1e-4, 1e-2, 1.0, 1e2, 1e6)]
    dist = [abs(v - lin) for v in vals]
    assert all(x >= y - 1e-15 for x, y in zip(dist, dist[1:]))
    assert dist[-1] < 1e-5 * dist[0]


def test_regularised_scheme_conserves_particle_number():
    """The zero-mass-flux walls stay exact with the regularisation (Eq. Ntot_def)."""
    o = CouetteOracle(N_R=24, ax1=(1, 6, 4), ax2=(0, 7, 4), Kn=0.5, u_in=0.3, R_out=1.5, weno_eps=1e-6)
    F = o.equilibrium(1, 0, 0, 1)
    m0 = o.mass(F)
    F = o.step(F, o.cfl_dt(0.5), 2000)
    assert abs(o.mass(F) / m0 - 1) <= 2000 * 2.2e-16


def test_equal_values_vanish_whatever_the_rounding():
    """A constant trailing stencil (c = d = e, the zeroth-order extrapolated ghosts of an
    open end) has sigma_3 = 0 exactly, although 3c - 4d + e can round to a residue: the
    regularisation must not apply there, so the flux is the Table weno limit."""
    rng = np.random.default_rng(8)
    hits = 0
    for _ in range(2000):
        a, b, c = rng.normal(size=3)
        if (3.0 * c - 4.0 * c) + c != 0.0:
            hits += 1
        assert weno5_eps(a, b, c, c, c, 1e-6) == weno5(a, b, c, c, c)
    assert hits > 0      # the rounding residue does occur for some values
