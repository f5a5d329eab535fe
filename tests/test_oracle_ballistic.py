"""Pins of the free-molecular Couette solution (Sec. V.E) in ``oracle/ballistic.py``:
the closed forms against the moments of the distribution function integrated directly,
the low-speed limit of Eq. bal_u_willis, the conservation laws of Eqs. TRph / Q_def, and
the mean density of Eq. ntot."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.ballistic import FreeMolecular

KEYS = ("n", "u", "T", "P", "TRR", "Tpp", "TRp", "qR", "qp")


@pytest.mark.parametrize("u_in", [0.5, 2.0])
def test_closed_forms_match_direct_integration(u_in):
    fm = FreeMolecular(1.0, 2.0, u_in, 1.0)
    for R in (1.02, 1.4, 1.98):
        a, b = fm.closed_form(R), fm.by_integration(R)
        assert abs(b["uR"]) < 1e-12                      # no net radial flow (Eq. n1n2)
        for k in KEYS:
            assert abs(a[k] - b[k]) <= 1e-10 * max(abs(b[k]), 1e-3), (R, k, a[k], b[k])


def test_trace_identity_and_conservation_laws():
    """3 n T = T^RR + T^phiphi + n T_w; R^2 T^Rphi and R (q^R + u T^Rphi) do not depend
    on R (Eqs. TRph, Q_def) -- from the direct integrals."""
    fm = FreeMolecular(1.0, 2.5, 1.5, 1.2)
    rows = [fm.by_integration(R) for R in (1.1, 1.7, 2.4)]
    for (R, b) in zip((1.1, 1.7, 2.4), rows):
        assert abs(3 * b["n"] * b["T"] - (b["TRR"] + b["Tpp"] + b["n"] * fm.T_w)) < 1e-12
    am = [R * R * b["TRp"] for R, b in zip((1.1, 1.7, 2.4), rows)]
    en = [R * (b["qR"] + b["u"] * b["TRp"]) for R, b in zip((1.1, 1.7, 2.4), rows)]
    assert max(am) - min(am) < 1e-10 * abs(am[0])
    assert max(en) - min(en) < 1e-10 * abs(en[0])


def test_mean_density():
    fm = FreeMolecular(1.0, 2.0, 1.0, 1.0)
    tot = integrate.quad(lambda R: fm.closed_form(R)["n"] * R, 1.0, 2.0, epsrel=1e-12)[0]
    assert abs(tot - 1.5) < 1e-10                        # Eq. ntot: mean density 1


def test_low_speed_limit_is_willis():
    """Eq. bal_u_willis: u^phi = (Omega R / pi)(theta_max - (R_in/R) sqrt(1 - R_in^2/R^2))
    up to O(Omega^3)."""
    u_in = 1e-3
    fm = FreeMolecular(1.0, 2.0, u_in, 1.0)
    for R in (1.1, 1.5, 1.9):
        th = math.asin(1.0 / R)
        willis = u_in * R / math.pi * (th - math.sqrt(1 - 1 / R ** 2) / R)
        assert abs(fm.closed_form(R)["u"] - willis) <= 1e-5 * willis
    assert abs(fm.n_w - 1.0) < 1e-5 and abs(fm.closed_form(1.5)["T"] - 1.0) < 1e-5
