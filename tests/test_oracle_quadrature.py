"""Pins of the oracle's velocity-space tables against facts fixed by the mathematics.

Sources: Sec. IV.B (Gauss-Hermite rules), Sec. IV.C and Appendix D (derivative
kernels), Sec. IV.D (equilibrium expansions) of arXiv:1708.05944.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import quadrature as q


@pytest.mark.parametrize("Q", [2, 3, 4, 5, 8, 11, 16, 20])
def test_full_range_matches_numpy_hermegauss(Q):
    """Full-range rule = numpy's probabilists' Gauss-Hermite rule, weights / sqrt(2 pi)."""
    x, w = np.polynomial.hermite_e.hermegauss(Q)
    ax = q.axis(0, Q, 0)
    assert np.allclose(ax.p, x, rtol=0, atol=1e-13 * max(1, abs(x).max()))
    assert np.allclose(ax.w, w / math.sqrt(2 * math.pi), rtol=1e-11, atol=0)
    assert abs(ax.w.sum() - 1.0) < 1e-14


def test_half_range_first_polynomials_closed_form():
    """h_0 = sqrt(2), h_1 = sqrt(2 pi/(pi-2)) (x - sqrt(2/pi)): orthonormalising 1 and x
    against omega on [0, inf) by hand."""
    h = q.half_range_coeffs_mp(3)
    assert abs(float(h[0][0]) - math.sqrt(2)) < 1e-15
    c = math.sqrt(2 * math.pi / (math.pi - 2))
    assert abs(float(h[1][1]) - c) < 1e-14
    assert abs(float(h[1][0]) + c * math.sqrt(2 / math.pi)) < 1e-14


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 8, 12, 16])
def test_half_range_gauss_exactness(Q):
    """The Q-point half-range rule integrates x^r omega exactly on [0, inf) for r <= 2Q-1
    (Gauss property) and not for r = 2Q; reference values by adaptive quadrature."""
    ax = q.axis(1, Q, 0)
    xp, wp = ax.p[:Q], ax.w[:Q]
    assert np.all(xp > 0) and np.allclose(ax.p[Q:], -xp, atol=0)
    for r in range(0, 2 * Q + 1):
        ref, _ = integrate.quad(lambda x: x ** r * math.exp(-x * x / 2) / math.sqrt(2 * math.pi), 0, np.inf,
                                epsabs=0, epsrel=1e-13, limit=200)
        got = float(np.sum(wp * xp ** r))
        if r <= 2 * Q - 1:
            assert abs(got - ref) <= 2e-12 * ref, (r, got, ref)
        else:
            # Gauss error for x^{2Q}: int omega pi_Q^2 with pi_Q monic, i.e. 1 / h_{QQ}^2
            hQQ = float(q.half_range_coeffs_mp(Q)[Q][Q])
            assert abs((ref - got) * hQQ ** 2 - 1.0) < 2e-3


@pytest.mark.parametrize("Q", [2, 3, 5, 8, 16])
def test_half_range_weight_formula_equals_christoffel(Q):
    """Eq. w_hh must equal the Christoffel weights 1 / sum_{l<Q} h_l(x_i)^2."""
    with mp.workdps(120):
        h = q.half_range_coeffs_mp(Q)
        x, w = q.half_range_mp(Q)
        for xi, wi in zip(x, w):
            chris = 1 / sum(q.hh_eval(h, l, xi) ** 2 for l in range(Q))
            assert abs(wi / chris - 1) < mp.mpf(10) ** -40


def test_half_range_nodes_brute_force_small_Q():
    """Q = 2 nodes from a float64 brute force (monic orthogonal polynomial from the 2x2
    moment system, roots by numpy) agree with the high-precision construction."""
    mu = [2 ** ((r - 1) / 2) * math.gamma((r + 1) / 2) / math.sqrt(2 * math.pi) for r in range(5)]
    # x^2 + c1 x + c0 orthogonal to 1 and x
    A = np.array([[mu[0], mu[1]], [mu[1], mu[2]]])
    c0, c1 = np.linalg.solve(A, -np.array([mu[2], mu[3]]))
    roots = np.sort(np.roots([1, c1, c0]).real)
    assert np.allclose(q.axis(1, 2, 0).p[:2], roots, atol=1e-12)


def _rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


@pytest.mark.parametrize("kind,Q", [(0, 3), (0, 4), (0, 5), (0, 16), (0, 20), (1, 2), (1, 4), (1, 8), (1, 16)])
def test_kernel_moment_identities(kind, Q):
    """For any f: sum_k p^s (K f)_k = -s sum_k p^{s-1} f_k and
    sum_k p^s (Kt f)_k = -s sum_k p^s f_k for s <= Q-1 (integration by parts of the
    projected derivatives, Appendix D); checked relative to the size of the terms."""
    ax = q.axis(kind, Q, 0)
    p = ax.p
    rng = np.random.default_rng(1234 + Q)
    f = rng.uniform(0.2, 1.0, ax.n_nodes) * ax.w
    Kf, Ktf = ax.K @ f, ax.Kt @ f
    for s in range(Q):
        scale = np.sum(np.abs(p) ** s * (np.abs(ax.K) @ np.abs(f))) + 1e-300
        lhs = np.sum(p ** s * Kf)
        rhs = -s * np.sum(p ** (s - 1) * f) if s > 0 else 0.0
        assert abs(lhs - rhs) <= 1e-12 * scale, ("K", s, lhs, rhs)
        scale = np.sum(np.abs(p) ** s * (np.abs(ax.Kt) @ np.abs(f))) + 1e-300
        lhs = np.sum(p ** s * Ktf)
        rhs = -s * np.sum(p ** s * f)
        assert abs(lhs - rhs) <= 1e-12 * scale, ("Kt", s, lhs, rhs)


@pytest.mark.parametrize("kind,Q", [(0, 4), (0, 5), (1, 4), (1, 8), (1, 16)])
def test_kernels_differentiate_the_maxwellian_exactly(kind, Q):
    """With f_k = w_k (the weighted standard Gaussian): df/dp = -p f, d(pf)/dp = (1-p^2) f."""
    ax = q.axis(kind, Q, 0)
    assert np.allclose(ax.K @ ax.w, -ax.p * ax.w, atol=1e-13, rtol=0)
    assert np.allclose(ax.Kt @ ax.w, (1 - ax.p ** 2) * ax.w, atol=1e-13, rtol=0)


def test_full_range_kernel_on_polynomial_times_gaussian():
    """f = omega (a + b p + c p^2) sampled as w_k(...): d/dp gives omega (b + 2cp - p(a+bp+cp^2))
    exactly while the degree stays below Q."""
    ax = q.axis(0, 6, 0)
    a, b, c = 0.7, -0.3, 0.25
    p, w = ax.p, ax.w
    f = w * (a + b * p + c * p * p)
    want = w * (b + 2 * c * p - p * (a + b * p + c * p * p))
    assert np.allclose(ax.K @ f, want, atol=1e-13)
    want_t = w * (a + 2 * b * p + 3 * c * p * p - p * p * (a + b * p + c * p * p))
    assert np.allclose(ax.Kt @ f, want_t, atol=1e-13)


def _full_moment(r, u, T):
    return q.gauss_moment_full(r, u, T)


@pytest.mark.parametrize("Q,N", [(4, 2), (5, 4), (16, 4), (20, 4)])
@pytest.mark.parametrize("u,T", [(0.0, 1.0), (0.3, 1.2), (-0.45, 0.8)])
def test_full_range_equilibrium_moments(Q, N, u, T):
    """Eq. eq_gak_H reproduces the Gaussian moments E[p^r], r <= N (Sec. IV.D)."""
    from oracle.couette import CouetteOracle
    o = CouetteOracle(N_R=3, ax1=(0, Q, N), ax2=(0, Q, N))
    fp, _ = o.feq(1.0, u, 0.0, T)
    g = fp.reshape(o.Q1, o.Q2).sum(axis=1)          # marginal over axis 2 = g1
    for r in range(N + 1):
        assert abs(np.sum(g * o.a1.p ** r) - _full_moment(r, u, T)) < 1e-12 * (1 + abs(_full_moment(r, u, T)))


@pytest.mark.parametrize("Q,N", [(4, 2), (4, 3), (8, 4), (16, 4)])
@pytest.mark.parametrize("u,T", [(0.0, 1.0), (0.3, 1.2), (-0.45, 0.8)])
def test_half_range_equilibrium_half_moments(Q, N, u, T):
    """Eq. eq_gak_hh reproduces the half-range moments int_0^inf p^r g and
    int_-inf^0 |p|^r g for r <= N; reference values by adaptive quadrature."""
    from oracle.couette import CouetteOracle
    o = CouetteOracle(N_R=3, ax1=(1, Q, N), ax2=(0, 4, 2))
    fp, _ = o.feq(1.0, u, 0.0, T)
    g = fp.reshape(o.Q1, o.Q2).sum(axis=1)
    gauss = lambda x: math.exp(-(x - u) ** 2 / (2 * T)) / math.sqrt(2 * math.pi * T)
    p = o.a1.p
    for r in range(N + 1):
        ref_p, _ = integrate.quad(lambda x: x ** r * gauss(x), 0, np.inf, epsabs=0, epsrel=1e-13)
        ref_m, _ = integrate.quad(lambda x: (-x) ** r * gauss(x), -np.inf, 0, epsabs=0, epsrel=1e-13)
        got_p = np.sum(g[:Q] * p[:Q] ** r)
        got_m = np.sum(g[Q:] * np.abs(p[Q:]) ** r)
        assert abs(got_p - ref_p) < 1e-11 * (1 + ref_p)
        assert abs(got_m - ref_m) < 1e-11 * (1 + ref_m)


def test_feq_reduced_temperature_relation():
    """f''_eq = T f'_eq (the line after Eq. feq_red) and the moments of f_eq give back
    (n, u, T) when N >= 2 on both axes."""
    from oracle.couette import CouetteOracle
    o = CouetteOracle(N_R=3, ax1=(1, 4, 3), ax2=(0, 5, 4))
    fp, fpp = o.feq(1.3, 0.2, -0.35, 1.1)
    assert np.allclose(fpp, 1.1 * fp, rtol=1e-15, atol=0)
    F = np.stack([np.tile(fp, (3, 1)), np.tile(fpp, (3, 1))])
    m = o.moments(F)
    assert np.allclose(m["n"], 1.3, rtol=1e-13)
    assert np.allclose(m["u1"], 0.2, atol=1e-13)
    assert np.allclose(m["u2"], -0.35, atol=1e-13)
    assert np.allclose(m["T"], 1.1, rtol=1e-13)
