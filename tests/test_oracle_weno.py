"""Pins of the oracle's epsilon-free WENO-5 (Sec. III.C of arXiv:1708.05944)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.couette import weno5, weno5_omega, weno5_sigma

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "weno_table.txt")


def _table():
    rows = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, *vals = line.split()
        rows[name] = [float(Fraction(v)) for v in vals]
    return rows


@pytest.mark.parametrize("name,sig", [
    ("all_equal", (0.7, 0.7, 0.7)), ("all_equal", (0.0, 0.0, 0.0)),
    ("s2=s3=0", (0.4, 0.0, 0.0)), ("s3=s1=0", (0.0, 2.0, 0.0)), ("s1=s2=0", (0.0, 0.0, 3.0)),
    ("s1=0", (0.0, 1.0, 5.0)), ("s2=0", (1.0, 0.0, 2.0)), ("s3=0", (9.0, 0.5, 0.0)),
])
def test_weights_match_paper_table(name, sig):
    """Every row of Table weno (tests/golden/weno_table.txt)."""
    assert np.allclose(weno5_omega(*sig), _table()[name], atol=1e-15)


def test_weights_generic_and_scale_invariant():
    """Generic case: omega_q proportional to delta_q / sigma_q^2, invariant when all sigma
    scale together (Eq. weno5_omega)."""
    w = weno5_omega(1.0, 2.0, 4.0)
    raw = np.array([0.1 / 1, 0.6 / 4, 0.3 / 16])
    assert np.allclose(w, raw / raw.sum(), rtol=1e-15)
    assert np.allclose(weno5_omega(1e-3, 2e-3, 4e-3), w, rtol=1e-14)


def test_constant_and_ghost_cases():
    """Constants are transported exactly; three equal upwind cells (the wall ghosts of
    Eq. weno_populate) give sigma_1 = 0 and the flux is the ghost value."""
    assert weno5(2.5, 2.5, 2.5, 2.5, 2.5) == pytest.approx(2.5, abs=4e-16)
    assert weno5(1.75, 1.75, 1.75, 0.3, 9.0) == pytest.approx(1.75, abs=1e-15)


def test_candidate_stencils_exact_for_quadratics():
    """Each candidate stencil is exact for quadratics in the cell-average sense: the
    averages of x^2 over unit cells centred at c = -2..2 are c^2 + 1/12, and every
    candidate (hence any convex combination) returns the point value 1/4 at x = 1/2."""
    avg = [c * c + 1.0 / 12 for c in (-2, -1, 0, 1, 2)]
    assert weno5(*avg) == pytest.approx(0.25, abs=1e-14)


def test_mirror_symmetry():
    """The V < 0 flux is the mirror image of the V > 0 one: weno5 on reversed data."""
    data = [0.3, 1.1, 0.7, 2.0, 1.4, 0.2]
    # face between data[2] and data[3]; upwind from the right uses (d5, d4, d3, d2, d1)
    right = weno5(data[5], data[4], data[3], data[2], data[1])
    rev = data[::-1]
    left_of_reversed = weno5(rev[0], rev[1], rev[2], rev[3], rev[4])
    assert right == left_of_reversed


def _deriv_error(N):
    """(F_{s+1/2} - F_{s-1/2})/h vs f'(x_s) for f = exp(x) on [0, 1] (no critical points),
    interior cells only; point values as in the finite-difference WENO of Eq. weno5_flux."""
    h = 1.0 / N
    x = (np.arange(-3, N + 3) + 0.5) * h
    f = np.exp(x)
    flux = [weno5(f[i - 2], f[i - 1], f[i], f[i + 1], f[i + 2]) for i in range(2, N + 4)]
    # flux[m] is the face right of cell index m+2 in x
    D = np.array([(flux[i + 1] - flux[i]) / h for i in range(N + 1)])
    xs = x[3:N + 4]
    err = np.abs(D - np.exp(xs))[3:-3]
    return err.max()


def test_fifth_order_on_smooth_data():
    """Constant-velocity advection is fifth order (Sec. III.E): errors fall ~32x per
    halving of h on smooth data without critical points."""
    e = [_deriv_error(N) for N in (20, 40, 80)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) > 4.5, (e, orders)


def _reconstruction(vals, centres):
    """Quadratic p(x) = al + be x + ga x^2 whose averages over the unit cells centred at
    `centres` equal `vals` (cell-average reconstruction; target cell [-1/2, 1/2])."""
    M = np.array([[1.0, m, m * m + 1.0 / 12] for m in centres])
    return np.linalg.solve(M, np.asarray(vals, dtype=float))


@pytest.mark.parametrize("seed", range(6))
def test_smoothness_indicators_and_flux_from_definition(seed):
    """Jiang-Shu definition of the smoothness indicators, independent of the printed
    closed form: sigma_q = int_{-1/2}^{1/2} (p_q')^2 + (p_q'')^2 dx for the quadratic p_q
    reconstructing stencil q, i.e. be^2 + (13/3) ga^2; candidate flux p_q(1/2).  The
    oracle's Eq. weno_sigma values and its flux (weights pinned by Table weno) must
    agree with this route."""
    rng = np.random.default_rng(seed)
    data = rng.uniform(-1, 2, 5) * (10.0 ** rng.integers(-12, 1))
    stencils = [((-2, -1, 0), data[0:3]), ((-1, 0, 1), data[1:4]), ((0, 1, 2), data[2:5])]
    sig, cand = [], []
    for centres, vals in stencils:
        al, be, ga = _reconstruction(vals, centres)
        sig.append(be * be + 13.0 / 3.0 * ga * ga)
        cand.append(al + be / 2 + ga / 4)
    got = weno5_sigma(*data)
    scale = max(sig)
    assert np.allclose(got, sig, rtol=1e-12, atol=1e-13 * scale)
    want = float(np.dot(weno5_omega(*sig), cand))
    assert weno5(*data) == pytest.approx(want, rel=1e-12, abs=1e-14 * np.abs(data).max())
