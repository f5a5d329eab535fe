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
* ``channel_512x128()``: the expanding channel of Sec. VI, 512 (xi) x 128 (lambda) cells,
  xi in [-4, 12], expansion ratio 2 over L = 4, HH(4;8) x H(4;16) (256 velocities),
  Kn = 0.05 with tau = Kn/(nT), reservoirs n = 1.1 / 0.9, T_w = 1.
* ``channel_sweep(B, seed)``: B channels drawn with numpy PCG64(seed): N_lambda =
  16 randint(4, 17), N_xi = 4 N_lambda, Kn = 10^U(-2, 0), r ~ U(1.5, 3); the p^lambda
  order grows with Kn: t = (log10 Kn + 2)/2, Q_lambda = 8 + round(8 t) (half range),
  Q_xi = 16 (full range), N = 4: 256 to 512 velocities.
"""
from __future__ import annotations

import numpy as np

from .vlb import VLB_TAU_AOKI, VLB_TAU_HYDRO, ChannelDesc, CouetteDesc

SWEEP_SEED = 20261203
CHANNEL_SWEEP_SEED = 3


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


# ---------------------------------------------------------------- learned warm start
# Training and held-out instances come from the sweep generator with their own seeds
# (1 and 2); the surrogate's inputs are position-normalised, so the training solves may
# use a coarser grid than the instances they warm-start.
SURROGATE_TRAIN_SEED, SURROGATE_HELDOUT_SEED = 1, 2


def surrogate_descs(B: int, seed: int, N_R: int | None = None, Kn_min: float = 0.0, Kn_max: float = np.inf):
    """Sweep instances of the given seed; N_R overrides the drawn grid size; instances
    with Kn outside [Kn_min, Kn_max] are skipped (drawn in order until B are kept)."""
    out, draw = [], max(B, 16)
    while len(out) < B:
        out = [d for d in couette_sweep(draw, seed) if Kn_min <= d.Kn <= Kn_max][:B]
        draw *= 2
    if N_R is not None:
        for d in out:
            d.N_R = int(N_R)
    return out


def mlp_init_params(width: int = 128, depth: int = 3, seed: int = 0, d_in: int = 4, d_out: int = 4):
    """Initial surrogate parameters, layer by layer W[fan_in][fan_out] then b[fan_out]:
    W ~ U(-a, a), a = sqrt(6 / (fan_in + fan_out)) (Glorot & Bengio 2010), b = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = [d_in] + [width] * depth + [d_out]
    parts = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts)


def epoch_orders(n: int, epochs: int, seed: int = 0):
    """One random permutation of range(n) per epoch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(epochs):
        yield rng.permutation(n).astype(np.int32)


# ---------------------------------------------------------------- expanding channel
def channel_512x128(Kn: float = 0.05) -> ChannelDesc:
    return ChannelDesc(N_lambda=128, N_xi=512, xi_in=-4.0, xi_out=12.0, r=2.0, L=4.0, ax1=(1, 8, 4), ax2=(0, 16, 4),
                       Kn=Kn, tau_model=VLB_TAU_HYDRO, n_in=1.1, n_out=0.9, T_w=1.0)


def channel_sweep(B: int = 64, seed: int = CHANNEL_SWEEP_SEED):
    rng = np.random.Generator(np.random.PCG64(seed))
    NL = 16 * rng.integers(4, 17, B)
    Kn = 10.0 ** rng.uniform(-2.0, 0.0, B)
    r = rng.uniform(1.5, 3.0, B)
    out = []
    for b in range(B):
        t = (np.log10(Kn[b]) + 2.0) / 2.0
        Ql = 8 + int(round(8 * t))
        out.append(ChannelDesc(N_lambda=int(NL[b]), N_xi=4 * int(NL[b]), xi_in=-4.0, xi_out=12.0, r=float(r[b]),
                               L=4.0, ax1=(1, Ql, 4), ax2=(0, 16, 4), Kn=float(Kn[b]), tau_model=VLB_TAU_HYDRO,
                               n_in=1.1, n_out=0.9, T_w=1.0))
    return out


CHANNEL_SURROGATE_TRAIN_SEED, CHANNEL_SURROGATE_HELDOUT_SEED = 11, 12
CHANNEL_SURROGATE_KN = (0.04, 0.25)
CHANNEL_SURROGATE_R = (1.5, 3.0)


def channel_surrogate_descs(B: int, seed: int, N_xi: int = 32, N_lambda: int = 8):
    """Reduced channel family of the learned channel warm start: Kn log-uniform in
    [0.04, 0.25] (tau = Kn/(nT); above Kn ~ 0.3 members of the family settle on a limit
    cycle at r ~ 1e-5 instead of a steady state), expansion ratio r uniform in [1.5, 3] over L = 4,
    xi in [-4, 12], HH(3;4) x H(4;8) = 64 velocities, reservoirs n 1.1 / 0.9, T_w = 1,
    regularised WENO weights (weno_eps = 1e-6), rest initial state."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.log10(CHANNEL_SURROGATE_KN[0]), np.log10(CHANNEL_SURROGATE_KN[1])
    Kn = 10.0 ** rng.uniform(lo, hi, B)
    r = rng.uniform(CHANNEL_SURROGATE_R[0], CHANNEL_SURROGATE_R[1], B)
    return [ChannelDesc(N_lambda=N_lambda, N_xi=N_xi, xi_in=-4.0, xi_out=12.0, r=float(r[b]), L=4.0, ax1=(1, 4, 3),
                        ax2=(0, 8, 4), Kn=float(Kn[b]), tau_model=VLB_TAU_HYDRO, n_in=1.1, n_out=0.9, T_w=1.0,
                        weno_eps=1e-6) for b in range(B)]
