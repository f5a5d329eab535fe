"""Seeded synthetic workloads (no method arithmetic here).

The paper measures on its own synthetic Couette set-ups (Sec. V); there is no dataset.
These generators produce instance descriptors with the shapes of those runs:

* ``single_couette()``: R_in = 1, R_out = 2, inner wall speed 0.1, T_w = 1, 64
  equidistant cells, HH(2;4) x H(2;4) (32 velocities), Kn = 0.1 with
  tau = Kn sqrt(pi/8)/n, CFL 0.5.
* ``couette_sweep(B, seed)``: B instances drawn with numpy PCG64(seed):
  Kn = 10^U(-2, 1), u_w ~ U(0.05, 0.5), beta = R_in/R_out ~ U(0.3, 0.8) with R_in = 1,
  N_R ~ randint(64, 513); quadrature orders grow with Kn:
  t = (log10 Kn + 2)/3, Q_R = 4 + round(12 t) (half range on p^R),
  Q_phi = 4 + round(16 t) (full range on p^phi), expansion order N = min(Q - 1, 4).
"""
from __future__ import annotations

import numpy as np

from .vlb import VLB_TAU_AOKI, CouetteDesc

SWEEP_SEED = 20261203


def single_couette(dt: float = 0.0) -> CouetteDesc:
    return CouetteDesc(R_in=1.0, R_out=2.0, N_R=64, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1,
                       tau_model=VLB_TAU_AOKI, dt=dt, cfl=0.5, u_in=0.1, T_in=1.0, u_out=0.0, T_out=1.0)


def sweep_params(B: int = 256, seed: int = SWEEP_SEED):
    """Raw draws of the sweep: list of dicts (Kn, u_w, beta, N_R, Q_R, Q_phi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Kn = 10.0 ** rng.uniform(-2.0, 1.0, B)
    uw = rng.uniform(0.05, 0.5, B)
    beta = rng.uniform(0.3, 0.8, B)
    NR = rng.integers(64, 513, B)
    out = []
    for b in range(B):
        t = (np.log10(Kn[b]) + 2.0) / 3.0
        QR = 4 + int(round(12 * t))
        Qp = 4 + int(round(16 * t))
        out.append(dict(Kn=float(Kn[b]), u_w=float(uw[b]), beta=float(beta[b]), N_R=int(NR[b]), Q_R=QR, Q_phi=Qp))
    return out


def couette_sweep(B: int = 256, seed: int = SWEEP_SEED, cfl: float = 0.5):
    descs = []
    for p in sweep_params(B, seed):
        descs.append(CouetteDesc(R_in=1.0, R_out=1.0 / p["beta"], N_R=p["N_R"],
                                 ax1=(1, p["Q_R"], min(p["Q_R"] - 1, 4)), ax2=(0, p["Q_phi"], min(p["Q_phi"] - 1, 4)),
                                 Kn=p["Kn"], tau_model=VLB_TAU_AOKI, dt=0.0, cfl=cfl, u_in=p["u_w"], T_in=1.0,
                                 u_out=0.0, T_out=1.0))
    return descs


def site_velocities(descs) -> int:
    """Sum over instances of cells x velocities (the unit of the throughput metric)."""
    tot = 0
    for d in descs:
        n1 = d.ax1[1] * (2 if d.ax1[0] == 1 else 1)
        n2 = d.ax2[1] * (2 if d.ax2[0] == 1 else 1)
        tot += d.N_R * n1 * n2
    return tot
