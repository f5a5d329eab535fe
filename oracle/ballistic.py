"""Free-molecular (ballistic) circular Couette flow, Sec. V.E (TEST INFRASTRUCTURE ONLY).

With no collisions, particles fly on straight lines between the cylinders.  The inner
cylinder (radius R_in, wall speed u_in = Omega_in R_in) and the outer one (R_out, at
rest) emit diffuse Maxwellians at the common wall temperature T_w with the same
emission density n_w (no net radial flux, Eq. n1n2); n_w is fixed by the mean density
(Eq. ntot: 2 pi int n R dR = pi (R_out^2 - R_in^2)).  At radius R a particle moving at
angle theta from the outward radial direction, |theta| < theta_max = arcsin(R_in / R),
comes from the inner cylinder (Eq. bal_f1), any other from the outer one (Eq. bal_f2).

Two independent routes to the profiles (m = k_B = 1):

* ``closed_form`` -- the paper's expressions: Eqs. bal_n, bal_u, bal_T (with the power of
  Rt in its last term read as in Eq. bal_u), bal_TRR, bal_Tpp, bal_TRp, bal_q, bal_Q (with
  Eq. Q_def), written with the integrals
  I_k = int_0^{Rt_in} zeta^(2k+1) e^(zeta^2) erf(zeta) / sqrt(1 - zeta^2 / Rt^2) d zeta
  evaluated by quadrature;
* ``by_integration`` -- the definition: moments of the distribution of Eqs. bal_f1 /
  bal_f2 integrated numerically over (p, theta), p_z analytically.

The tests pin ``closed_form`` to ``by_integration``; the solver's ballistic steady state
is then compared with ``closed_form``.
"""
from __future__ import annotations

import math

import mpmath as mp
from scipy import integrate


class FreeMolecular:
    def __init__(self, R_in: float = 1.0, R_out: float = 2.0, u_in: float = 1.0, T_w: float = 1.0):
        self.R_in, self.R_out, self.u_in, self.T_w = float(R_in), float(R_out), float(u_in), float(T_w)
        self.Omega = self.u_in / self.R_in
        # n_w from the mean density (Eq. ntot); n / n_w depends on R only
        area = integrate.quad(lambda R: self._n_over_nw(R) * R, self.R_in, self.R_out, epsabs=0, epsrel=1e-13,
                              limit=200)[0]
        self.n_w = (self.R_out ** 2 - self.R_in ** 2) / (2.0 * area)

    # ------------------------------------------------------------------ helpers
    def _rt(self, R: float):
        return self.Omega * R / math.sqrt(2.0 * self.T_w)

    def _I(self, k: int, R: float) -> float:
        """I_k(Rt) of the closed forms (the integrable endpoint singularity at R = R_in
        is handled by the tanh-sinh rule)."""
        Rt = mp.mpf(self._rt(R))
        Rt_in = mp.mpf(self.u_in / math.sqrt(2.0 * self.T_w))
        with mp.workdps(30):
            f = lambda z: z ** (2 * k + 1) * mp.exp(z * z) * mp.erf(z) / mp.sqrt(1 - (z / Rt) ** 2)
            return float(mp.quad(f, [0, Rt_in]))

    def _n_over_nw(self, R: float) -> float:
        Rt = self._rt(R)
        Rt_in = self.u_in / math.sqrt(2.0 * self.T_w)
        th = math.asin(self.R_in / R)
        E = math.exp(-Rt_in ** 2)
        return 1.0 - th / math.pi + E * (th / math.pi + self._I(0, R) / (Rt * math.sqrt(math.pi)))

    # ------------------------------------------------------------------ closed forms
    def closed_form(self, R: float) -> dict:
        """n, u^phi, T, P, T^RR, T^phiphi, T^Rphi, q^R, q^phi at radius R from the
        paper's expressions (Sec. V.E.2)."""
        Tw, nw, Ri = self.T_w, self.n_w, self.R_in
        Rt = self._rt(R)
        Rt_in = self.u_in / math.sqrt(2.0 * Tw)
        th = math.asin(Ri / R)
        c = math.cos(th)
        E = math.exp(-Rt_in ** 2)
        sp = math.sqrt(math.pi)
        I0, I1, I2 = (self._I(k, R) for k in range(3))
        n = nw * (1.0 - th / math.pi + E * (th / math.pi + I0 / (Rt * sp)))                      # Eq. bal_n
        u = nw * self.Omega * R * E / (2 * math.pi * n) * (th - Ri / R * c + sp / Rt ** 3 * (I0 + 2 * I1))   # Eq. bal_u
        TRR = (nw * Tw / math.pi * E * (Ri / (4 * R) * (4 + 2 * Rt_in ** 2 - Rt ** 2) * c + 0.25 * (4 + Rt ** 2) * th
                                        + sp / Rt ** 3 * (3 * Rt ** 2 * I0 + (2 * Rt ** 2 - 3) * I1 - 2 * I2))
               + nw * Tw * (1 - th / math.pi - math.sin(2 * th) / (2 * math.pi)))                  # Eq. bal_TRR
        Tpp = (nw * Tw / math.pi * E * (-Ri / (4 * R) * (4 + 2 * Rt_in ** 2 + 3 * Rt ** 2) * c
                                        + 0.25 * (4 + 3 * Rt ** 2) * th + sp / Rt ** 3 * (3 * I1 + 2 * I2))
               + nw * Tw * (1 - th / math.pi + math.sin(2 * th) / (2 * math.pi)) - n * u * u)     # Eq. bal_Tpp
        # Eq. bal_T; its last term carries sqrt(pi) / Rt^3 as in Eq. bal_u (the printed
        # power is 1, which breaks 3 n T = T^RR + T^phiphi + n T_w and the direct integral)
        T = (Tw - u * u / 3.0
             + nw * Tw * Rt ** 2 / (3 * math.pi * n) * E * (th - Ri / R * c + sp / Rt ** 3 * (I0 + 2 * I1)))
        TRp = nw * Tw / sp * Rt_in * Ri ** 2 / R ** 2                                              # Eq. bal_TRp
        Q = nw * Ri * Tw ** 1.5 / math.sqrt(2 * math.pi) * Rt_in ** 2                            # Eq. bal_Q
        qR = Q / R - u * TRp                                                                       # Eq. Q_def
        m21_03 = (nw * Tw ** 1.5 * Rt * E / (4 * math.pi * math.sqrt(2.0))
                  * (th * (10 + 3 * Rt ** 2) - Ri / R * (10 + 2 * Rt_in ** 2 + 3 * Rt ** 2) * c
                     + 2 * sp / Rt ** 3 * (3 * I0 + 12 * I1 + 4 * I2)))
        qp = m21_03 + 0.5 * n * Tw * u - u * Tpp - 0.5 * n * u ** 3 - 1.5 * n * u * T              # Eq. bal_q
        return dict(n=n, u=u, T=T, P=n * T, TRR=TRR, Tpp=Tpp, TRp=TRp, qR=qR, qp=qp)

    # ------------------------------------------------------------------ by integration
    def by_integration(self, R: float) -> dict:
        """The same moments from the distribution function itself (Eqs. bal_f1, bal_f2),
        integrated over the momentum plane (p, theta) with p_z done analytically."""
        Tw, nw = self.T_w, self.n_w
        th_m = math.asin(self.R_in / R)
        A = nw / (2 * math.pi * Tw)        # p_z-integrated Maxwellian prefactor
        uin2 = self.u_in ** 2
        OR = self.Omega * R

        def f(p, th):
            if abs(th) < th_m:
                return A * math.exp(-(p * p + uin2 - 2 * p * OR * math.sin(th)) / (2 * Tw))
            return A * math.exp(-p * p / (2 * Tw))

        pmax = 12.0 * math.sqrt(Tw) + 2.0 * self.u_in * R / self.R_in

        def mom(g):
            tot = 0.0
            for a, b in ((-math.pi, -th_m), (-th_m, th_m), (th_m, math.pi)):
                tot += integrate.dblquad(lambda p, th: g(p, th) * f(p, th) * p, a, b, 0.0, pmax,
                                         epsabs=1e-14, epsrel=1e-12)[0]
            return tot

        n = mom(lambda p, th: 1.0)
        u = mom(lambda p, th: p * math.sin(th)) / n
        uR = mom(lambda p, th: p * math.cos(th)) / n
        PRR = mom(lambda p, th: (p * math.cos(th)) ** 2)
        Ppp = mom(lambda p, th: (p * math.sin(th) - u) ** 2)
        PRp = mom(lambda p, th: p * math.cos(th) * (p * math.sin(th) - u))
        T = (PRR + Ppp + n * Tw) / (3 * n)
        c2 = lambda p, th: (p * math.cos(th)) ** 2 + (p * math.sin(th) - u) ** 2
        qR = 0.5 * mom(lambda p, th: c2(p, th) * p * math.cos(th))
        qp = 0.5 * mom(lambda p, th: c2(p, th) * (p * math.sin(th) - u))
        return dict(n=n, u=u, uR=uR, T=T, P=n * T, TRR=PRR, Tpp=Ppp, TRp=PRp, qR=qR, qp=qp)
