"""Cartesian-split ("CLB") form of the expanding channel, Sec. VI.G (TEST INFRASTRUCTURE ONLY).

The momentum space keeps its Cartesian components (p^x, p^y) -- ax1 the p^x axis
(across the channel), ax2 the p^y axis (along it) -- so there are no force terms; only
the advection velocities carry the geometry (Eq. canalie_coord_beq_cons):

    d_t f + d_lambda(V^lambda f) + d_chi(V^xi f) = -(f - f_eq) / tau,
    V^lambda = (p^x - lambda phi' p^y) / (1 + phi),   V^xi = (1 + phi) p^y.

Everything else follows the vielbein channel of ``oracle.channel`` (same grid, cells,
equilibrium expansions of Sec. IV.D in the axes' own variables, BGK, RK3, reservoir
ends) with these choices:

* V^lambda at the lambda faces of column p uses the discrete metric
  a_p = (1 + phi_p)(phi_{p+1/2} - phi_{p-1/2}) / dchi_p in place of phi'_p, so that the flux
  differences of a uniform state cancel exactly (free-stream preservation);
* walls (lambda = -1, +1): a population is wall-bound or emitted by the sign of V^lambda at
  the wall face (Sec. VI.G: the half-planes depend on position); emitted ghosts are
  n_w f_eq(1, 0, T_w) with n_w of Eq. canalie_coord_nw (f' only; f'' ghosts carry T_w);
  wall-bound ghosts continue the quadratic through the three cells next to the wall
  (Eq. extrapol, and 10 F1 - 15 F2 + 6 F3 for the third ghost, which faces whose own
  V^lambda has the other sign reach);
* ends: reservoirs as for the vielbein channel (entering populations, p^y > 0 at the
  inlet and < 0 at the outlet, see three ghosts at f_eq(n_in / n_out, 0, T_w); leaving
  ones a zeroth-order extrapolation), or the flow-rate ends of Sec. VI.C.1-2: every row s
  carries Q_s = 3 Q0 / (H (1 + phi)) (1 - 4 lambda_s^2 / H^2) through both end faces, the
  entering ghosts at n_s f_eq(1, (0, Q_s), T_w) (Cartesian components here), n_s from the
  row balance with the leaving populations of the end cell;
* the half channel (lambda in [0, 1]) mirrors p^x at the centreline: ghost -1-m of
  population (i, j) is cell m's population of the mirrored p^x node (Sec. VI.C.3).

WENO-5 face values come from the pinned C routine of ``oracle.couette`` (epsilon-free
weights of Sec. III.C), one call per population and face.
"""
from __future__ import annotations

import numpy as np

from .channel import ChannelOracle
from .couette import weno5, weno5_eps


class ClbOracle(ChannelOracle):
    def __init__(self, NL=8, NX=12, ax1=(1, 4, 2), ax2=(1, 4, 2), **kw):
        super().__init__(NL=NL, NX=NX, ax1=ax1, ax2=ax2, **kw)
        self.weno_eps = kw.get("weno_eps", 0.0)
        # discrete metric a_p (free-stream preserving form of phi')
        self.metric = (1.0 + self.phi_c) * np.diff(self.phi_f) / self.dchi
        self.px = np.repeat(self.a1.p, self.Q2)
        self.py = np.tile(self.a2.p, self.Q1)
        Qh = self.a1.Q                                        # p^x -> -p^x on the half-range axis
        self.mirror = np.array([((i + Qh) % (2 * Qh)) * self.Q2 + j for i in range(self.Q1) for j in range(self.Q2)])

    def cartesian_velocity(self, m):
        """The moments of the Cartesian-split populations are Cartesian already."""
        return m["u1"], m["u2"]

    def _w(self, a, b, c, d, e):
        return weno5(a, b, c, d, e) if self.weno_eps == 0.0 else weno5_eps(a, b, c, d, e, self.weno_eps)

    def _face(self, G, c, v, k):
        """WENO value at the face between extended cells c and c + 1 (index into G, which
        starts three ghosts before cell 0) for velocity k, upwinded by the sign of v."""
        if v > 0:
            return self._w(G[c - 2, k], G[c - 1, k], G[c, k], G[c + 1, k], G[c + 2, k])
        return self._w(G[c + 3, k], G[c + 2, k], G[c + 1, k], G[c, k], G[c - 1, k])

    def _vlam(self, lam, p):
        return (self.px - lam * self.metric[p] * self.py) / (1.0 + self.phi_c[p])

    def wall_density(self, F):
        """n_w of both walls of every column (Eq. canalie_coord_nw), [NX][2] (lower, upper)."""
        F = np.asarray(F).reshape(2, self.NX, self.NL, self.NV)
        fw = self.feq(1.0, 0.0, 0.0, self.T_w)[0]
        out = np.empty((self.NX, 2))
        NL = self.NL
        for p in range(self.NX):
            for side, lam in ((0, self.lam_f[0]), (1, self.lam_f[-1])):
                if side == 0 and self.half:
                    out[p, 0] = 0.0                           # specular centreline, no wall
                    continue
                v = self._vlam(lam, p)
                bound = v < 0 if side == 0 else v > 0
                G = self._column(F[0], p, None, None)
                num = den = 0.0
                c = 2 if side == 0 else NL + 2          # extended index of the cell below the wall face
                for k in range(self.NV):
                    if bound[k]:
                        num += v[k] * self._face(G, c, v[k], k)
                    elif (v[k] < 0 if side == 1 else v[k] > 0):
                        den += v[k] * fw[k]
                out[p, side] = -num / den
        return out

    def _column(self, Fd, p, nw, fw):
        """Column p of one distribution with three ghosts at each wall, [NL + 6][NV];
        nw = (lower, upper) n_w and fw the unit emitted Maxwellian (None: wall-bound
        extrapolation for every velocity, as needed to evaluate the wall-bound flux)."""
        NL = self.NL
        G = np.zeros((NL + 6, self.NV))
        G[3:NL + 3] = Fd[p]
        lo = self._vlam(self.lam_f[0], p)
        hi = self._vlam(self.lam_f[-1], p)
        F1, F2, F3 = Fd[p, 0], Fd[p, 1], Fd[p, 2]
        ext_lo = [10 * F1 - 15 * F2 + 6 * F3, 6 * F1 - 8 * F2 + 3 * F3, 3 * F1 - 3 * F2 + F3]   # cells -3, -2, -1
        G1, G2, G3 = Fd[p, NL - 1], Fd[p, NL - 2], Fd[p, NL - 3]
        ext_hi = [3 * G1 - 3 * G2 + G3, 6 * G1 - 8 * G2 + 3 * G3, 10 * G1 - 15 * G2 + 6 * G3]   # cells NL .. NL+2
        for q in range(3):
            G[q] = ext_lo[q]
            G[NL + 3 + q] = ext_hi[q]
            if nw is not None:
                G[q] = np.where(lo > 0, nw[0] * fw, G[q])            # emitted upward from the lower wall
                G[NL + 3 + q] = np.where(hi < 0, nw[1] * fw, G[NL + 3 + q])
            if self.half:                                     # cell q - 3 = -1 - m mirrors cell m
                G[q] = Fd[p, 2 - q][self.mirror]
        return G

    def wall_flux(self, F):
        """Total f' flux sum_k V^lambda F_face through the lower and upper wall face of every
        column with the ghosts L uses, [NX][2]; zero by the construction of n_w."""
        F = np.asarray(F, dtype=np.float64).reshape(2, self.NX, self.NL, self.NV)
        nw = self.wall_density(F)
        fw = self.feq(1.0, 0.0, 0.0, self.T_w)[0]
        out = np.empty((self.NX, 2))
        for p in range(self.NX):
            G = self._column(F[0], p, nw[p], fw)
            for side, (f, lam) in enumerate(((0, self.lam_f[0]), (self.NL, self.lam_f[-1]))):
                v = self._vlam(lam, p)
                out[p, side] = sum(v[k] * self._face(G, f + 2, v[k], k) for k in range(self.NV))
        return out

    def L(self, F):
        """L[F] of the Cartesian-split channel; returns (L, n_w [NX][2])."""
        F = np.asarray(F, dtype=np.float64).reshape(2, self.NX, self.NL, self.NV)
        NL, NX, NV = self.NL, self.NX, self.NV
        m = self.moments(F)
        Feq = self.equilibrium(m["n"], m["u1"], m["u2"], m["T"])
        if self.tau_model == 0:
            tau = self.Kn * np.sqrt(np.pi / 8) / m["n"]
        elif self.tau_model == 1:
            tau = self.Kn / (m["n"] * m["T"])
        else:
            tau = self.Kn / m["n"]
        out = -(F - Feq) / tau[None, :, :, None]
        nw = self.wall_density(F)
        fw = self.feq(1.0, 0.0, 0.0, self.T_w)
        fin = self.feq(self.n_in, 0.0, 0.0, self.T_w)
        fout = self.feq(self.n_out, 0.0, 0.0, self.T_w)
        for d in range(2):
            wall = fw[d]
            # lambda direction, column by column
            for p in range(NX):
                G = self._column(F[d], p, nw[p], wall)
                flux = np.empty((NL + 1, NV))                   # face s - 1/2, s = 0..NL
                for f in range(NL + 1):
                    v = self._vlam(self.lam_f[f], p)
                    for k in range(NV):
                        flux[f, k] = v[k] * self._face(G, f + 2, v[k], k)
                out[d, p] -= (flux[1:] - flux[:-1]) / self.dlam[:, None]
            # xi direction, row by row
            for s in range(NL):
                H = np.zeros((NX + 6, NV))
                H[3:NX + 3] = F[d, :, s]
                gin, gout = (fin[d], fout[d]) if self.ends == 0 else self._end_ghosts(F, s, d)
                for q in range(3):
                    H[q] = np.where(self.py > 0, gin, F[d, 0, s])
                    H[NX + 3 + q] = np.where(self.py < 0, gout, F[d, NX - 1, s])
                flux = np.empty((NX + 1, NV))
                for f in range(NX + 1):
                    v = (1.0 + self.phi_f[f]) * self.py
                    for k in range(NV):
                        flux[f, k] = v[k] * self._face(H, f + 2, v[k], k)
                out[d, :, s] -= (flux[1:] - flux[:-1]) / self.dchi[:, None]
        return out, nw

    def _end_ghosts(self, F, s, d):
        """Entering ghosts of row s at the inlet and outlet for the flow-rate ends."""
        out = []
        for e, face, end in ((0, 0, 0), (1, self.NX, self.NX - 1)):
            Q = self.profile(face)[s]
            f1 = self.feq(1.0, 0.0, Q, self.T_w)
            entering = self.py > 0 if e == 0 else self.py < 0
            leave = np.sum(np.where(entering, 0.0, F[0, end, s] * self.py))
            dens = np.sum(np.where(entering, f1[0] * self.py, 0.0))
            out.append((Q - leave) / dens * f1[d])
        return out

    def end_flow(self, F):
        """Flow rate sum_k p^y F_face of f' of every row at the inlet and outlet faces, [2][NL],
        with the ghosts L uses."""
        F = np.asarray(F, dtype=np.float64).reshape(2, self.NX, self.NL, self.NV)
        fin = self.feq(self.n_in, 0.0, 0.0, self.T_w)[0]
        fout = self.feq(self.n_out, 0.0, 0.0, self.T_w)[0]
        out = np.empty((2, self.NL))
        for s in range(self.NL):
            H = np.zeros((self.NX + 6, self.NV))
            H[3:self.NX + 3] = F[0, :, s]
            gin, gout = (fin, fout) if self.ends == 0 else self._end_ghosts(F, s, 0)
            for q in range(3):
                H[q] = np.where(self.py > 0, gin, F[0, 0, s])
                H[self.NX + 3 + q] = np.where(self.py < 0, gout, F[0, self.NX - 1, s])
            for e, f in ((0, 0), (1, self.NX)):
                out[e, s] = sum(self.py[k] * self._face(H, f + 2, self.py[k], k) for k in range(self.NV))
        return out

    def step(self, F, dt: float, nsteps: int = 1):
        """SSP-RK3 steps (Eq. rk3) of the Cartesian-split channel."""
        F = np.asarray(F, dtype=np.float64).reshape(2, self.NX, self.NL, self.NV).copy()
        for _ in range(nsteps):
            F1 = F + dt * self.L(F)[0]
            F2 = 0.75 * F + 0.25 * F1 + 0.25 * dt * self.L(F1)[0]
            F = F / 3.0 + 2.0 / 3.0 * F2 + 2.0 / 3.0 * dt * self.L(F2)[0]
        return F

    def cfl_dt(self, cfl: float = 0.5) -> float:
        best = 0.0
        for p in range(self.NX):
            vx = np.abs((1.0 + self.phi_f[[p, p + 1]])[:, None] * self.py[None, :]).max()
            for s in range(self.NL):
                vl = max(np.abs(self._vlam(self.lam_f[s], p)).max(), np.abs(self._vlam(self.lam_f[s + 1], p)).max())
                best = max(best, vl / self.dlam[s] + vx / self.dchi[p])
        return cfl / best
