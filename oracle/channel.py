"""Python front end of the plain-C expanding-channel oracle (TEST INFRASTRUCTURE ONLY).

Builds ``channel_oracle.c`` (which includes the Couette oracle's velocity-set code)
with gcc -O2 -ffp-contract=off, fills its parameter struct with the mpmath tables of
``oracle.quadrature`` and the channel geometry computed here in 40-digit arithmetic:

* wall 1 + phi(xi) = 1 + (r - 1) [1 + tanh(4 xi / L - 2)] / 2 (inlet half-width 1,
  outlet half-width r, the tanh profile of Eq. canalie_phi rescaled to these
  asymptotes), phi' its derivative;
* chi(xi) = xi + (r - 1) [xi + (L/4) ln cosh(4 xi / L - 2)] / 2, so d chi = (1 + phi) d xi
  (Eq. chi_canalie), cell widths dchi_p = chi(xi_{p+1/2}) - chi(xi_{p-1/2});
* lambda in [-1, 1] (the full channel width, walls at both ends) on equal cells, xi on
  equal cells in [xi_in, xi_out]; or, with ``half``, lambda in [0, 1] with a specular
  centreline (Sec. VI.C.3).  ``ends = 1`` replaces the reservoirs by the flow-rate
  profile of Sec. VI.C.1-2 with flow rate Q0 through half of the cross-section.

State layout: float64 F[2][NX][NL][NV] (f' then f''), NV = Q1*Q2, k = i*Q2 + j with i
the p^lambda node (axis 1) and j the p^xi node (axis 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import mpmath as mp
import numpy as np

from . import quadrature as quad
from .couette import TAU_AOKI, TAU_HYDRO, TAU_KN, _Params  # noqa: F401  (shared oracle struct)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "channel_oracle.c")
_DEP = os.path.join(_HERE, "couette_oracle.c")
_LIB = os.path.join(_HERE, "_channel_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_DEP))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-Wall",
                               "-Werror=sequence-point", "-Werror=unused-value", "-I", _HERE, "-shared", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_DP = ctypes.POINTER(ctypes.c_double)


class _CParams(ctypes.Structure):
    _fields_ = ([("vs", _Params), ("NL", ctypes.c_int), ("NX", ctypes.c_int)]
                + [(n, _DP) for n in ("Kt1", "K2", "lam_f", "phi_c", "dphi_c", "phi_f", "dphi_f", "dchi")]
                + [(n, ctypes.c_double) for n in ("n_in", "n_out", "T_w")]
                + [("half", ctypes.c_int), ("ends", ctypes.c_int), ("Q0", ctypes.c_double)])


def lib():
    global _lib
    with _lock:
        if _lib is None:
            _lib = ctypes.CDLL(build())
            dp = ctypes.POINTER(ctypes.c_double)
            _lib.oracle_channel_L.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
            _lib.oracle_channel_L2.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp]
            _lib.oracle_channel_rk3.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_long]
            _lib.oracle_feq.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 4 + [dp, dp]
        return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def wall_phi(xi, r: float, L: float = 4.0, d: int = 0):
    """phi(xi) (d = 0) or phi'(xi) (d = 1) of the expanding wall, 40-digit arithmetic."""
    with mp.workdps(40):
        z = 4 * mp.mpf(xi) / L - 2
        if d == 0:
            return float((r - 1) * (1 + mp.tanh(z)) / 2)
        return float((r - 1) * 2 / L * mp.sech(z) ** 2)


def wall_chi(xi, r: float, L: float = 4.0):
    with mp.workdps(40):
        x = mp.mpf(xi)
        return (x + (r - 1) * (x + mp.mpf(L) / 4 * mp.log(mp.cosh(4 * x / L - 2))) / 2)


def d3(f, x, axis):
    """First derivative of samples f at the (possibly unequally spaced) nodes x along
    `axis`, by the three-point Lagrange formulas of Sec. VI.F (vorticity): centred on the
    nodes 1 .. n-2, one-sided second order on the first and last node (the last-node
    formula with the sign that makes it exact for constants).  Exact for quadratics."""
    f = np.moveaxis(np.asarray(f, dtype=np.float64), axis, 0)
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 3:
        raise ValueError("need three nodes")
    out = np.empty_like(f)
    for s in range(1, n - 1):
        hm, hp = x[s] - x[s - 1], x[s + 1] - x[s]
        out[s] = (hm * f[s + 1] / (hp * (hp + hm)) + (hp - hm) * f[s] / (hp * hm)
                  - hp * f[s - 1] / ((hp + hm) * hm))
    a, b, c = x[0], x[1], x[2]
    out[0] = (-(b + c - 2 * a) * f[0] / ((b - a) * (c - a)) + (c - a) * f[1] / ((b - a) * (c - b))
              - (b - a) * f[2] / ((c - a) * (c - b)))
    a, b, c = x[n - 1], x[n - 2], x[n - 3]
    out[n - 1] = ((2 * a - b - c) * f[n - 1] / ((a - b) * (a - c)) - (a - c) * f[n - 2] / ((a - b) * (b - c))
                  + (a - b) * f[n - 3] / ((a - c) * (b - c)))
    return np.moveaxis(out, 0, axis)


class ChannelOracle:
    """One expanding channel: NL cells across lambda in [-1, 1], NX cells along
    xi in [xi_in, xi_out], expansion ratio r over length L, reservoir densities n_in /
    n_out, walls at rest at T_w; ax1 (p^lambda, half range for the walls) and ax2
    (p^xi) as (kind, Q, N)."""

    def __init__(self, NL=8, NX=12, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.05, tau_model=TAU_HYDRO, r=2.0, L=4.0,
                 xi_in=-4.0, xi_out=12.0, n_in=1.1, n_out=0.9, T_w=1.0, weno_eps=0.0, half=False, ends=0, Q0=0.0,
                 A=0.0):
        if NL < (3 if half else 6) or NX < 3:
            raise ValueError("need at least 6 lambda cells (two walls; 3 for the half channel) and 3 xi cells")
        self.a1, self.a2 = quad.axis(*ax1), quad.axis(*ax2)
        self.Q1, self.Q2 = self.a1.n_nodes, self.a2.n_nodes
        self.NV = self.Q1 * self.Q2
        self.NL, self.NX = NL, NX
        self.half, self.ends, self.Q0 = bool(half), int(ends), float(Q0)
        # equal cells, or equal cells in eta with lambda = tanh(eta) / A (Eq. canalie_stretch,
        # H / 2 = 1), eta over [0, artanh A] (half channel) or [-artanh A, artanh A]
        t = [(s / NL) if half else (-1.0 + 2.0 * s / NL) for s in range(NL + 1)]
        with mp.workdps(40):
            self.lam_f = np.array([float(mp.tanh(x * mp.atanh(A)) / A) if A > 0 else x for x in t])
        self.lam_c = 0.5 * (self.lam_f[1:] + self.lam_f[:-1])
        self.dlam = np.diff(self.lam_f)
        self.xi_f = np.array([xi_in + (xi_out - xi_in) * p / NX for p in range(NX + 1)])
        self.xi_c = 0.5 * (self.xi_f[1:] + self.xi_f[:-1])
        self.phi_c = np.array([wall_phi(x, r, L) for x in self.xi_c])
        self.dphi_c = np.array([wall_phi(x, r, L, 1) for x in self.xi_c])
        self.phi_f = np.array([wall_phi(x, r, L) for x in self.xi_f])
        self.dphi_f = np.array([wall_phi(x, r, L, 1) for x in self.xi_f])
        chi = [wall_chi(x, r, L) for x in self.xi_f]
        self.dchi = np.array([float(chi[p + 1] - chi[p]) for p in range(NX)])
        self.Kn, self.tau_model = Kn, tau_model
        self.n_in, self.n_out, self.T_w = n_in, n_out, T_w
        self._keep = {}
        vs = _Params()
        vs.NR, vs.Q1, vs.Q2 = 0, self.Q1, self.Q2
        vs.kind1, vs.kind2, vs.N1, vs.N2 = self.a1.kind, self.a2.kind, self.a1.N, self.a2.N
        vs.Qh1, vs.Qh2 = self.a1.Q, self.a2.Q
        arrays = dict(p1=self.a1.p, w1=self.a1.w, p2=self.a2.p, w2=self.a2.w, B1=self.a1.basis, B2=self.a2.basis,
                      K1=self.a1.K, Kt2=self.a2.Kt)
        for name, arr in arrays.items():
            arr = np.ascontiguousarray(arr, dtype=np.float64)
            self._keep[name] = arr
            setattr(vs, name, _ptr(arr))
        vs.Kn, vs.tau_model, vs.weno_eps = Kn, tau_model, weno_eps
        vs.u_in = vs.u_out = 0.0
        vs.T_in = vs.T_out = T_w
        P = _CParams()
        P.vs = vs
        P.NL, P.NX = NL, NX
        extra = dict(Kt1=self.a1.Kt, K2=self.a2.K, lam_f=self.lam_f, phi_c=self.phi_c, dphi_c=self.dphi_c,
                     phi_f=self.phi_f, dphi_f=self.dphi_f, dchi=self.dchi)
        for name, arr in extra.items():
            arr = np.ascontiguousarray(arr, dtype=np.float64)
            self._keep["c_" + name] = arr
            setattr(P, name, _ptr(arr))
        P.n_in, P.n_out, P.T_w = n_in, n_out, T_w
        P.half, P.ends, P.Q0 = int(bool(half)), int(ends), float(Q0)
        self._P = P
        self.W = np.outer(self.a1.w, self.a2.w).ravel()
        self.vol = np.outer(self.dchi, self.dlam)          # [NX][NL] cell volumes dchi_p dlambda_s

    def L(self, F):
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(2, self.NX, self.NL, self.NV)
        out = np.empty_like(F)
        flux = np.empty(self.NX + 1)
        nw = np.empty((self.NX, 2))
        lib().oracle_channel_L(ctypes.byref(self._P), _ptr(F), _ptr(out), _ptr(flux), _ptr(nw))
        return out, flux, nw

    def end_flow(self, F):
        """Flow rate sum_k p^y F_face of f' of every lambda row at the inlet and outlet
        faces, [2][NL]."""
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(2, self.NX, self.NL, self.NV)
        out = np.empty_like(F)
        rf = np.empty((2, self.NL))
        lib().oracle_channel_L2(ctypes.byref(self._P), _ptr(F), _ptr(out), None, None, _ptr(rf))
        return rf

    def profile(self, face: int):
        """Prescribed flow rate of every lambda row at xi face 0 or NX (ends = 1)."""
        H = 2.0
        return 3.0 * self.Q0 / (H * (1.0 + self.phi_f[face])) * (1.0 - 4.0 * self.lam_c ** 2 / H ** 2)

    def step(self, F, dt: float, nsteps: int = 1):
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(2, self.NX, self.NL, self.NV).copy()
        lib().oracle_channel_rk3(ctypes.byref(self._P), _ptr(F), dt, nsteps)
        return F

    def feq(self, n, u1, u2, T):
        fe = np.empty(2 * self.NV)
        lib().oracle_feq(ctypes.byref(self._P.vs), n, u1, u2, T, _ptr(fe), _ptr(fe[self.NV:]))
        return fe.reshape(2, self.NV)

    def equilibrium(self, n, u1, u2, T):
        """Local-equilibrium state of per-cell fields (scalars or [NX][NL] arrays)."""
        shp = (self.NX, self.NL)
        n, u1, u2, T = (np.broadcast_to(np.asarray(x, dtype=np.float64), shp) for x in (n, u1, u2, T))
        F = np.empty((2, self.NX, self.NL, self.NV))
        for p in range(self.NX):
            for s in range(self.NL):
                fe = self.feq(n[p, s], u1[p, s], u2[p, s], T[p, s])
                F[0, p, s], F[1, p, s] = fe[0], fe[1]
        return F

    def moments(self, F):
        F = np.asarray(F).reshape(2, self.NX, self.NL, self.NV)
        p1 = np.repeat(self.a1.p, self.Q2)
        p2 = np.tile(self.a2.p, self.Q1)
        n = F[0].sum(-1)
        u1 = (F[0] * p1).sum(-1) / n
        u2 = (F[0] * p2).sum(-1) / n
        e = ((p1 ** 2 + p2 ** 2) * F[0]).sum(-1) + F[1].sum(-1)
        T = (e - n * (u1 ** 2 + u2 ** 2)) / (3 * n)
        return dict(n=n, u1=u1, u2=u2, T=T)

    def flow_fields(self, F):
        """Diagnostics of Sec. VI.D and VI.F (plain numpy from the cell moments):
        ux, uy: Cartesian velocity from the triad components (Eq. canalie_u), [NX][NL];
        P = n T, [NX][NL];
        psi: stream function on the lambda faces, [NX][NL + 1], from rho u_y = -d psi / dx
          (Eq. canalie_psi) integrated across each xi column with dx = (1 + phi) d lambda,
          psi = 0 on the centreline (lambda = 0);
        omega: vorticity (Eq. canalie_vorti) at the cell centres, both derivatives by the
          three-point formulas of d3;
        Pw: pressure on the lambda faces 0 and NL (the lower wall, or the centreline of the
          half channel; the upper wall) by linear extrapolation from the two outermost cells
          (the construction before Eq. canalie_wall_pressure), [2][NX]."""
        m = self.moments(F)
        n, T = m["n"], m["T"]
        lam = np.broadcast_to(self.lam_c[None, :], n.shape)
        a = lam * self.dphi_c[:, None]
        ux, uy = self.cartesian_velocity(m)
        P = n * T
        # stream function: d psi = -rho u_y dx across each xi column, dx = (1 + phi) d lambda;
        # the running sum from the lower face, shifted to vanish at lambda = 0 (linear inside
        # the cell holding it when that is not a face)
        width = (1.0 + self.phi_c)[:, None] * self.dlam[None, :]
        cum = np.concatenate([np.zeros((self.NX, 1)), np.cumsum(n * uy * width, axis=1)], axis=1)
        s0 = min(int(np.searchsorted(self.lam_f, 0.0, side="right")) - 1, self.NL - 1)
        frac = (0.0 - self.lam_f[s0]) / self.dlam[s0]
        psi = -(cum - ((1 - frac) * cum[:, s0:s0 + 1] + frac * cum[:, s0 + 1:s0 + 2]))
        omega = (-d3(ux, self.xi_c, 0) + (d3(uy, self.lam_c, 1) + a * d3(ux, self.lam_c, 1))
                 / (1.0 + self.phi_c)[:, None])
        # wall pressure: the line through the two outermost cell values, at the face; the
        # ratio of the physical offsets x = lambda (1 + phi) equals that of the lambda offsets
        Pw = np.empty((2, self.NX))
        for side, (e, i1, i2) in enumerate(((0, 0, 1), (self.NL, self.NL - 1, self.NL - 2))):
            lw, l1, l2 = self.lam_f[e], self.lam_c[i1], self.lam_c[i2]
            Pw[side] = ((lw - l2) * P[:, i1] - (lw - l1) * P[:, i2]) / (l1 - l2)
        return dict(ux=ux, uy=uy, P=P, psi=psi, omega=omega, Pw=Pw)

    def cartesian_velocity(self, m):
        """(u^x, u^y) of every cell from the triad components (Eq. canalie_u)."""
        lam = np.broadcast_to(self.lam_c[None, :], m["n"].shape)
        a = lam * self.dphi_c[:, None]
        c = 1.0 / np.sqrt(1.0 + a * a)
        return (m["u1"] + a * m["u2"]) * c, (m["u2"] - a * m["u1"]) * c

    def mass(self, F):
        F = np.asarray(F).reshape(2, self.NX, self.NL, self.NV)
        return float((self.vol * F[0].sum(-1)).sum())

    def residual(self, F_new, F_old, dt):
        a = np.asarray(F_new).reshape(2, self.NX, self.NL, self.NV)
        b = np.asarray(F_old).reshape(2, self.NX, self.NL, self.NV)
        w = self.vol[None, :, :, None] / self.W[None, None, None, :]
        return float(np.sqrt((w * (a - b) ** 2).sum() / (w * b ** 2).sum()) / dt)

    def cfl_dt(self, cfl: float = 0.5) -> float:
        """cfl / max over cells and velocities of |V^lambda| / dlambda + |V^xi| / dchi."""
        best = 0.0
        p1, p2 = self.a1.p, self.a2.p
        for p in range(self.NX):
            for s in range(self.NL):
                lam = self.lam_c[s]
                vl = np.sqrt(1 + max(self.lam_f[s] ** 2, self.lam_f[s + 1] ** 2) * self.dphi_c[p] ** 2) / (
                    1 + self.phi_c[p]) * np.abs(p1).max() / self.dlam[s]
                vx = 0.0
                for f in (p, p + 1):
                    a = lam * self.dphi_f[f]
                    vx = max(vx, (1 + self.phi_f[f]) * (np.abs(p2).max() + abs(a) * np.abs(p1).max())
                             / np.sqrt(1 + a * a))
                best = max(best, vl + vx / self.dchi[p])
        return cfl / best
