"""Python front end of the plain-C Couette oracle (TEST INFRASTRUCTURE ONLY).

Builds ``couette_oracle.c`` with gcc (-O2 -ffp-contract=off, no fast-math), fills
its parameter struct with the mpmath tables of ``oracle.quadrature`` and the grid of
Sec. V.C.1 (cell-centred radii; optional tanh stretching, Sec. III.B, Eqs. eta_def
and eta_inout), and exposes L[F], RK3 steps, moments, mass and the steady-state
residual.

State layout: float64 array F[2][NR][NV] (f' then f''), NV = Q1*Q2, k = i*Q2 + j.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

from . import quadrature as quad

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "couette_oracle.c")
_LIB = os.path.join(_HERE, "_couette_oracle.so")
_lock = threading.Lock()
_lib = None

TAU_AOKI, TAU_HYDRO, TAU_KN = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle shared object next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-Wall",
                               "-Werror=sequence-point", "-Werror=unused-value", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            _lib = ctypes.CDLL(build())
            dp = ctypes.POINTER(ctypes.c_double)
            _lib.oracle_couette_L.argtypes = [ctypes.c_void_p, dp, dp, dp]
            _lib.oracle_couette_rk3.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_long]
            _lib.oracle_feq.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 4 + [dp, dp]
            _lib.oracle_weno5.argtypes = [ctypes.c_double] * 5
            _lib.oracle_weno5.restype = ctypes.c_double
            _lib.oracle_weno5_eps.argtypes = [ctypes.c_double] * 6
            _lib.oracle_weno5_eps.restype = ctypes.c_double
            _lib.oracle_weno5_omega.argtypes = [ctypes.c_double] * 3 + [dp]
            _lib.oracle_weno5_sigma.argtypes = [ctypes.c_double] * 5 + [dp]
        return _lib


class _Params(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int) for n in ("NR", "Q1", "Q2", "kind1", "kind2", "N1", "N2", "Qh1", "Qh2")]
                + [(n, ctypes.POINTER(ctypes.c_double)) for n in
                   ("p1", "w1", "p2", "w2", "B1", "B2", "K1", "Kt2", "Rf", "dchi", "Gam")]
                + [("Kn", ctypes.c_double), ("tau_model", ctypes.c_int)]
                + [(n, ctypes.c_double) for n in ("u_in", "T_in", "u_out", "T_out", "weno_eps")]
                + [("form", ctypes.c_int)]
                + [(n, ctypes.POINTER(ctypes.c_double)) for n in ("sqg", "ef")]
                + [(n, ctypes.c_double) for n in ("deta", "sqg_in", "sqg_out")])


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def weno5(a, b, c, d, e) -> float:
    """The oracle's epsilon-free WENO-5 flux (upwind cell c), Sec. III.C."""
    return lib().oracle_weno5(a, b, c, d, e)


def weno5_eps(a, b, c, d, e, eps) -> float:
    """Regularised WENO-5 flux (an extension; eps = 0 is the paper's scheme): when no
    indicator vanishes exactly, each gets eps * mean(a^2 .. e^2) added."""
    return lib().oracle_weno5_eps(a, b, c, d, e, eps)


def weno5_omega(s1, s2, s3) -> np.ndarray:
    """Normalised WENO-5 weights for smoothness indicators (s1, s2, s3), Eq. weno5_omega
    with the limits of Table weno."""
    w = np.zeros(3)
    lib().oracle_weno5_omega(s1, s2, s3, _ptr(w))
    return w


def weno5_sigma(a, b, c, d, e) -> np.ndarray:
    """Smoothness indicators of Eq. weno_sigma for upwind-ordered cells (a, b, c, d, e)."""
    s = np.zeros(3)
    lib().oracle_weno5_sigma(a, b, c, d, e, _ptr(s))
    return s


def couette_faces(R_in: float, R_out: float, N_R: int, A: float = 0.0, delta: float = 0.5) -> np.ndarray:
    """Face radii R_{s-1/2}, s = 1..N_R+1.  A = 0: equidistant (Sec. V.C.1);
    0 < A < 1: equidistant in eta with R(eta) of Eq. eta_def, range Eq. eta_inout."""
    s = np.arange(N_R + 1, dtype=np.float64)
    if A == 0.0:
        return R_in + s / N_R * (R_out - R_in)
    A0 = max(delta, 1.0 - delta)
    eta_l = -math.atanh(A * delta / A0)
    eta_r = math.atanh(A * (1.0 - delta) / A0)
    eta = eta_l + s / N_R * (eta_r - eta_l)
    R = R_in + (R_out - R_in) * (delta + A0 / A * np.tanh(eta))
    R[0], R[-1] = R_in, R_out
    return R


def ftilde_metric(R_in: float, R_out: float, N_R: int, A: float = 0.0, delta: float = 0.5):
    """Metric of the f-tilde formulation on the grid of couette_faces: sqrt(g) = R R'(eta)
    at the cell centres (eta_s = midpoint of the cell in eta), e_eta^eta = 1/R'(eta) at the
    faces, the cell width in eta, and sqrt(g) at the two walls (Sec. V.A, Eq.
    boltz_couette_str_cons with R(eta) of Eq. eta_def).  Equal cells: eta = R, R' = 1."""
    s = np.arange(N_R + 1, dtype=np.float64)
    if A == 0.0:
        Rf = R_in + s / N_R * (R_out - R_in)
        return 0.5 * (Rf[1:] + Rf[:-1]), np.ones(N_R + 1), (R_out - R_in) / N_R, R_in, R_out
    A0 = max(delta, 1.0 - delta)
    eta_l = -math.atanh(A * delta / A0)
    eta_r = math.atanh(A * (1.0 - delta) / A0)
    deta = (eta_r - eta_l) / N_R
    R = lambda eta: R_in + (R_out - R_in) * (delta + A0 / A * np.tanh(eta))
    dR = lambda eta: (R_out - R_in) * A0 / (A * np.cosh(eta) ** 2)
    etac = eta_l + (np.arange(N_R) + 0.5) * deta
    etaf = eta_l + s * deta
    return R(etac) * dR(etac), 1.0 / dR(etaf), deta, R_in * dR(eta_l), R_out * dR(eta_r)


class CouetteOracle:
    """One circular-Couette instance: R_in < R < R_out, inner wall speed u_in, outer u_out.

    ax1 / ax2 are (kind, Q, N) for the radial and azimuthal momentum axes
    (kind 0 = full-range H, 1 = half-range HH), e.g. HH(2;4) x H(2;4) is
    ax1=(1, 4, 2), ax2=(0, 4, 2).  weno_eps > 0 selects the regularised WENO weights
    (an extension for reaching steady states; 0 is the paper's epsilon-free scheme).
    form = 1 selects the f-tilde formulation (the advective flux reconstructed from
    sqrt(g) f, Sec. III Eq. boltz_cons), kept for the paper's comparison with the chi form
    (Sec. V.C.2); the state is f in both forms."""

    def __init__(self, R_in=1.0, R_out=2.0, N_R=64, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1,
                 tau_model=TAU_AOKI, u_in=0.1, T_in=1.0, u_out=0.0, T_out=1.0, A=0.0, delta=0.5,
                 weno_eps=0.0, form=0):
        if N_R < 3:
            raise ValueError("need at least 3 cells (wall extrapolation uses 3)")
        self.a1, self.a2 = quad.axis(*ax1), quad.axis(*ax2)
        self.Q1, self.Q2 = self.a1.n_nodes, self.a2.n_nodes
        self.NV = self.Q1 * self.Q2
        self.NR = N_R
        self.Rf = couette_faces(R_in, R_out, N_R, A, delta)
        self.Rc = 0.5 * (self.Rf[1:] + self.Rf[:-1])
        self.dchi = 0.5 * (self.Rf[1:] ** 2 - self.Rf[:-1] ** 2)
        self.Gam = 2.0 / (self.Rf[1:] + self.Rf[:-1])
        self.Kn, self.tau_model = Kn, tau_model
        self.walls = (u_in, T_in, u_out, T_out)
        self._keep = {}
        self.form = form
        self.sqg, self.ef, self.deta, sqg_in, sqg_out = ftilde_metric(R_in, R_out, N_R, A, delta)
        arrays = dict(p1=self.a1.p, w1=self.a1.w, p2=self.a2.p, w2=self.a2.w,
                      B1=self.a1.basis, B2=self.a2.basis, K1=self.a1.K, Kt2=self.a2.Kt,
                      Rf=self.Rf, dchi=self.dchi, Gam=self.Gam, sqg=self.sqg, ef=self.ef)
        P = _Params()
        P.NR, P.Q1, P.Q2 = N_R, self.Q1, self.Q2
        P.kind1, P.kind2, P.N1, P.N2 = self.a1.kind, self.a2.kind, self.a1.N, self.a2.N
        P.Qh1, P.Qh2 = self.a1.Q, self.a2.Q
        for name, arr in arrays.items():
            arr = np.ascontiguousarray(arr, dtype=np.float64)
            self._keep[name] = arr
            setattr(P, name, _ptr(arr))
        P.Kn, P.tau_model = Kn, tau_model
        P.u_in, P.T_in, P.u_out, P.T_out = u_in, T_in, u_out, T_out
        P.weno_eps = weno_eps
        P.form = form
        P.deta, P.sqg_in, P.sqg_out = self.deta, sqg_in, sqg_out
        self._P = P
        self.W = np.outer(self.a1.w, self.a2.w).ravel()      # quadrature weight per velocity

    # ------------------------------------------------------------------ core
    def L(self, F: np.ndarray):
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(2, self.NR, self.NV)
        out = np.empty_like(F)
        nw = np.zeros(2)
        lib().oracle_couette_L(ctypes.byref(self._P), _ptr(F), _ptr(out), _ptr(nw))
        return out, nw

    def step(self, F: np.ndarray, dt: float, nsteps: int = 1) -> np.ndarray:
        F = np.array(F, dtype=np.float64, order="C").reshape(2, self.NR, self.NV)
        lib().oracle_couette_rk3(ctypes.byref(self._P), _ptr(F), dt, nsteps)
        return F

    def feq(self, n, u1, u2, T):
        fp = np.empty(self.NV)
        fpp = np.empty(self.NV)
        lib().oracle_feq(ctypes.byref(self._P), n, u1, u2, T, _ptr(fp), _ptr(fpp))
        return fp, fpp

    def equilibrium(self, n, u1, u2, T) -> np.ndarray:
        """State with f' = f'_eq(n_s, u_s, T_s), f'' = T_s f'_eq at every cell."""
        bc = lambda x: np.broadcast_to(np.asarray(x, dtype=np.float64), (self.NR,))
        n, u1, u2, T = map(bc, (n, u1, u2, T))
        F = np.empty((2, self.NR, self.NV))
        for s in range(self.NR):
            F[0, s], F[1, s] = self.feq(n[s], u1[s], u2[s], T[s])
        return F

    # ------------------------------------------------------------------ diagnostics
    def moments(self, F: np.ndarray) -> dict:
        """n, u^R, u^phi, T, T^{R phi}, q^R, q^phi per cell (Eqs. macro_red), m = 1."""
        F = np.asarray(F).reshape(2, self.NR, self.Q1, self.Q2)
        fp, fpp = F[0], F[1]
        p1 = self.a1.p[None, :, None]
        p2 = self.a2.p[None, None, :]
        n = fp.sum(axis=(1, 2))
        u1 = (p1 * fp).sum(axis=(1, 2)) / n
        u2 = (p2 * fp).sum(axis=(1, 2)) / n
        x1 = p1 - u1[:, None, None]
        x2 = p2 - u2[:, None, None]
        xi2 = x1 ** 2 + x2 ** 2
        T = ((xi2 * fp).sum(axis=(1, 2)) + fpp.sum(axis=(1, 2))) / (3 * n)
        T12 = (x1 * x2 * fp).sum(axis=(1, 2))
        heat = 0.5 * (xi2 * fp + fpp)
        q1 = (heat * x1).sum(axis=(1, 2))
        q2 = (heat * x2).sum(axis=(1, 2))
        return dict(n=n, u1=u1, u2=u2, T=T, T12=T12, q1=q1, q2=q2)

    def mass(self, F: np.ndarray) -> float:
        """N_tot per unit height and per radian: sum_s dchi_s n_s (Eq. Ntot_def, chi form)."""
        F = np.asarray(F).reshape(2, self.NR, self.NV)
        return float((self.dchi * F[0].sum(axis=1)).sum())

    def residual(self, F_new: np.ndarray, F_old: np.ndarray, dt: float) -> float:
        """r = ||F_new - F_old||_W / (dt ||F_old||_W) with
        ||F||_W^2 = sum_s dchi_s sum_k (f'^2 + f''^2)/W_k."""
        a = np.asarray(F_new).reshape(2, self.NR, self.NV)
        b = np.asarray(F_old).reshape(2, self.NR, self.NV)
        wts = self.dchi[None, :, None] / self.W[None, None, :]
        num = ((a - b) ** 2 * wts).sum()
        den = (b ** 2 * wts).sum()
        return math.sqrt(num / den) / dt

    def cfl_dt(self, cfl: float = 0.5) -> float:
        """dt = CFL * min_s dchi_s / (max(R_{s+-1/2}) max_k |p^R_k|)."""
        pmax = np.abs(self.a1.p).max()
        return float(cfl * np.min(self.dchi / (self.Rf[1:] * pmax)))
