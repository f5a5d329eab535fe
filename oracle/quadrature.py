"""Velocity-space tables of the mixed-quadrature LB models, in arbitrary precision.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Everything here is written from the paper's Sec. IV (LB models) and Appendix D:

* full-range Gauss-Hermite (Sec. IV.B, Eq. w_H): nodes are the roots of the
  probabilists' Hermite polynomial He_Q, weights Q!/He_{Q+1}(x)^2 (they sum to 1);
* half-range Gauss-Hermite (Sec. IV.B, Eqs. hh_roots, w_hh, hh_a, hh_exp): the
  polynomials h_l are orthonormal on [0, inf) with respect to
  omega(x) = exp(-x^2/2)/sqrt(2 pi), leading coefficient positive.  The paper never
  states the normalisation; we read it as orthonormal because the kernels of
  Eqs. df_K_hh / dfp_K_hh carry no factorials.
  Nodes are the Q positive roots of h_Q, mirrored to the negative semi-axis, and
  the weights follow Eq. w_hh;
* momentum-derivative kernels (Sec. IV.C, Eqs. df_K_H, df_K_hh, dfp_K_H,
  dfp_K_hh; derivations in Appendix D);
* equilibrium basis tables used by Eqs. eq_gak_H and eq_gak_hh (Sec. IV.D):
  He_l(p_k) for full-range axes and Phi^N_s(|p_k|) (Eq. Phi_def) for half-range axes.

All arithmetic is mpmath at a working precision that grows with Q; results are
rounded to float64 only when handed out.  The half-range polynomials come from a
Cholesky factorisation of the exact Hankel moment matrix, which is ill-conditioned
in float64 but harmless at 80+ digits.
"""
from __future__ import annotations

import functools
import math

import mpmath as mp
import numpy as np

KIND_H = 0    # full-range Gauss-Hermite axis
KIND_HH = 1   # half-range Gauss-Hermite axis


def _dps(Q: int) -> int:
    return 60 + 4 * Q


# ----------------------------------------------------------------------------- full range
def he_values(n_max: int, x):
    """[He_0(x), ..., He_{n_max}(x)] for the probabilists' Hermite polynomials
    (orthogonal with weight omega, norm l!; Appendix D.1)."""
    out = [mp.mpf(1)]
    if n_max >= 1:
        out.append(mp.mpf(x))
    for n in range(1, n_max):
        out.append(x * out[n] - n * out[n - 1])
    return out


def _he_coeffs(n: int):
    """Integer coefficients of He_n, lowest power first."""
    c_prev, c = [1], [0, 1]
    if n == 0:
        return c_prev
    for k in range(1, n):
        nxt = [0] * (k + 2)
        for i, a in enumerate(c):
            nxt[i + 1] += a
        for i, a in enumerate(c_prev):
            nxt[i] -= k * a
        c_prev, c = c, nxt
    return c


@functools.lru_cache(maxsize=None)
def full_range_mp(Q: int):
    """Nodes (ascending) and weights of the order-Q full-range rule, Eq. w_H."""
    with mp.workdps(_dps(Q)):
        coeffs = _he_coeffs(Q)
        roots = mp.polyroots(list(reversed(coeffs)), maxsteps=400, extraprec=400)
        nodes = sorted(mp.re(r) for r in roots)
        fact = mp.factorial(Q)
        weights = [fact / he_values(Q + 1, x)[Q + 1] ** 2 for x in nodes]
        return nodes, weights


# ----------------------------------------------------------------------------- half range
def half_moment(r: int):
    """int_0^inf x^r omega(x) dx = 2^{(r-1)/2} Gamma((r+1)/2) / sqrt(2 pi)."""
    return mp.power(2, mp.mpf(r - 1) / 2) * mp.gamma(mp.mpf(r + 1) / 2) / mp.sqrt(2 * mp.pi)


@functools.lru_cache(maxsize=None)
def half_range_coeffs_mp(L: int):
    """Matrix h[l][s] (l, s = 0..L) of monomial coefficients of the orthonormal
    half-range polynomials h_l(x) = sum_s h[l][s] x^s (Eq. hh_exp)."""
    with mp.workdps(_dps(L)):
        H = mp.matrix(L + 1, L + 1)
        for a in range(L + 1):
            for b in range(L + 1):
                H[a, b] = half_moment(a + b)
        C = mp.cholesky(H)          # H = C C^T, C lower triangular
        P = mp.inverse(C)           # rows of C^{-1}: orthonormal coefficient vectors
        return [[P[l, s] if s <= l else mp.mpf(0) for s in range(L + 1)] for l in range(L + 1)]


def hh_eval(coeffs, l: int, x):
    return mp.polyval(list(reversed(coeffs[l][: l + 1])), x)


@functools.lru_cache(maxsize=None)
def half_range_mp(Q: int):
    """Positive nodes (ascending) and weights of the order-Q half-range rule
    (Eqs. hh_roots and w_hh)."""
    with mp.workdps(_dps(Q)):
        h = half_range_coeffs_mp(Q)
        roots = mp.polyroots(list(reversed(h[Q][: Q + 1])), maxsteps=800, extraprec=800)
        nodes = sorted(mp.re(r) for r in roots)
        a_Qm1 = h[Q][Q] / h[Q - 1][Q - 1]                       # Eq. hh_a with l = Q-1
        hQ0_sq = h[Q][0] ** 2
        weights = []
        for x in nodes:
            hqm1 = hh_eval(h, Q - 1, x)
            weights.append(x * a_Qm1 ** 2 / (hqm1 ** 2 * (x + hQ0_sq / mp.sqrt(2 * mp.pi))))
        return nodes, weights


# ----------------------------------------------------------------------------- axes
class Axis:
    """One momentum axis: kind (KIND_H / KIND_HH), order Q, f_eq expansion order N.

    Node ordering (Sec. IV.B): full range -> the Q roots of He_Q ascending;
    half range -> the Q positive roots ascending, then their mirrors -p_1..-p_Q.
    """

    def __init__(self, kind: int, Q: int, N: int):
        if kind not in (KIND_H, KIND_HH):
            raise ValueError("axis kind must be 0 (H) or 1 (HH)")
        if Q < 1 or not (0 <= N < Q):
            raise ValueError("need Q >= 1 and 0 <= N < Q (Eq. norder_limit)")
        self.kind, self.Q, self.N = kind, Q, N
        self.n_nodes = Q if kind == KIND_H else 2 * Q
        with mp.workdps(_dps(Q)):
            if kind == KIND_H:
                x, w = full_range_mp(Q)
                self._p = list(x)
                self._w = list(w)
            else:
                x, w = half_range_mp(Q)
                self._p = list(x) + [-v for v in x]
                self._w = list(w) + list(w)
        self.p = np.array([float(v) for v in self._p])
        self.w = np.array([float(v) for v in self._w])

    def sign(self, k: int) -> int:
        return 1 if k < self.Q else -1

    # ---- kernels of Sec. IV.C -------------------------------------------------------
    @functools.cached_property
    def K(self) -> np.ndarray:
        """Matrix of d/dp (Eq. df_K_H for full range, Eq. df_K_hh for half range)."""
        return self._kernel(tilde=False)

    @functools.cached_property
    def Kt(self) -> np.ndarray:
        """Matrix of d(p .)/dp (Eq. dfp_K_H, Eq. dfp_K_hh)."""
        return self._kernel(tilde=True)

    def _kernel(self, tilde: bool) -> np.ndarray:
        Q, n = self.Q, self.n_nodes
        with mp.workdps(_dps(Q)):
            M = [[mp.mpf(0)] * n for _ in range(n)]
            if self.kind == KIND_H:
                He = [he_values(Q + 1, x) for x in self._p]
                for k in range(n):
                    for kp in range(n):
                        acc = mp.mpf(0)
                        if not tilde:                       # Eq. df_K_H
                            for l in range(Q):
                                acc += He[k][l + 1] * He[kp][l] / mp.factorial(l)
                        else:                               # Eq. dfp_K_H
                            for l in range(Q - 1):
                                lower = l * He[kp][l - 1] if l >= 1 else mp.mpf(0)
                                acc += He[k][l + 1] * (He[kp][l + 1] + lower) / mp.factorial(l)
                        M[k][kp] = -self._w[k] * acc
            else:
                h = half_range_coeffs_mp(Q)
                absx = [abs(v) for v in self._p]
                hv = [[hh_eval(h, l, x) for l in range(Q + 1)] for x in absx]
                h0 = [h[l][0] for l in range(Q + 1)]
                a = [h[l + 1][l + 1] / h[l][l] for l in range(Q)]   # Eq. hh_a
                s2pi = mp.sqrt(2 * mp.pi)
                # Phi^Q_0(x) = sum_{l=0}^{Q} h_{l,0} h_l(x)   (Eq. Phi_def)
                phi0 = [sum(h0[l] * hv[k][l] for l in range(Q + 1)) for k in range(n)]
                for k in range(n):
                    sk = self.sign(k)
                    for kp in range(n):
                        skp = self.sign(kp)
                        same = (1 + sk * skp) // 2
                        if not tilde:                       # Eq. df_K_hh
                            acc = mp.mpf(0)
                            if same:
                                for l in range(Q - 1):
                                    inner = h0[l] / s2pi * sum(h0[s] * hv[k][s] for s in range(l + 1, Q))
                                    inner -= h[l][l] / h[l + 1][l + 1] * hv[k][l + 1]
                                    acc += hv[kp][l] * inner
                            acc -= phi0[k] * phi0[kp] / (2 * s2pi)
                            M[k][kp] = self._w[k] * sk * acc
                        else:                               # Eq. dfp_K_hh
                            acc = mp.mpf(0)
                            if same:
                                for l in range(Q):
                                    term = l * hv[kp][l]
                                    if l >= 1:
                                        term += (h0[l] ** 2 + h0[l - 1] ** 2) / (a[l - 1] * s2pi) * hv[kp][l - 1]
                                    if l >= 2:
                                        term += hv[kp][l - 2] / (a[l - 1] * a[l - 2])
                                    acc += hv[k][l] * term
                            M[k][kp] = -self._w[k] * acc
            return np.array([[float(v) for v in row] for row in M])

    # ---- equilibrium basis of Sec. IV.D ----------------------------------------------
    @functools.cached_property
    def basis(self) -> np.ndarray:
        """[n_nodes][N+1] table: He_l(p_k) (full range) or Phi^N_s(|p_k|) (half range)."""
        N = self.N
        with mp.workdps(_dps(self.Q)):
            if self.kind == KIND_H:
                rows = [he_values(max(N, 1), x)[: N + 1] for x in self._p]
            else:
                h = half_range_coeffs_mp(max(self.Q, N))
                rows = []
                for x in self._p:
                    ax = abs(x)
                    rows.append([sum(h[l][s] * hh_eval(h, l, ax) for l in range(s, N + 1))
                                 for s in range(N + 1)])
            return np.array([[float(v) for v in r] for r in rows])


@functools.lru_cache(maxsize=None)
def axis(kind: int, Q: int, N: int) -> Axis:
    return Axis(kind, Q, N)


def gauss_moment_full(r: int, u: float, T: float) -> float:
    """E[p^r] for p ~ Normal(u, T) (closed form via the binomial expansion)."""
    s = 0.0
    for k in range(0, r + 1, 2):
        s += math.comb(r, k) * u ** (r - k) * T ** (k // 2) * _double_factorial(k - 1)
    return s


def _double_factorial(n: int) -> int:
    return 1 if n <= 0 else n * _double_factorial(n - 2)
