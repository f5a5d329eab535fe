"""Pins of the expanding-channel oracle (oracle/channel.py, Sec. VI of arXiv:1708.05944)
against facts it does not compute itself: exact stationarity of the rest state in a
curved channel (the purpose of the discrete connection coefficients of Sec. VI.A),
particle-number balance against the end fluxes for arbitrary states (zero wall flux,
Eq. nw; telescoping fluxes; mass-conserving force kernels), mirror symmetry across the
centreline, and the equality of the particle flux through every cross-section at
steady state."""
import numpy as np
import pytest

from oracle.channel import ChannelOracle, wall_chi, wall_phi


def _perturbed(o, seed, amp=0.15):
    rng = np.random.default_rng(seed)
    X, S = np.meshgrid(o.xi_c, o.lam_c, indexing="ij")
    F = o.equilibrium(1 + 0.1 * np.sin(X) * np.cos(2 * S), 0.05 * np.sin(3 * S), 0.2 * np.cos(S) * (1 - S ** 2),
                      1 + 0.05 * np.cos(X + S))
    return F * rng.uniform(1 - amp, 1 + amp, F.shape)


def test_geometry_closed_forms():
    """phi -> 0 upstream and r - 1 downstream; d chi / d xi = 1 + phi (Eq. chi_canalie)."""
    assert abs(wall_phi(-40.0, 2.0)) < 1e-30 and abs(wall_phi(40.0, 2.0) - 1.0) < 1e-30
    for x in (-3.0, 0.5, 1.7, 6.0):
        h = 1e-6
        dchi = float(wall_chi(x + h, 2.0) - wall_chi(x - h, 2.0)) / (2 * h)
        assert dchi == pytest.approx(1 + wall_phi(x, 2.0), rel=1e-9)
        dphi = (wall_phi(x + h, 2.0) - wall_phi(x - h, 2.0)) / (2 * h)
        assert dphi == pytest.approx(wall_phi(x, 2.0, d=1), rel=1e-7, abs=1e-12)


@pytest.mark.parametrize("kw", [
    dict(NL=8, NX=10, ax1=(1, 4, 2), ax2=(0, 4, 2), r=2.0),
    dict(NL=6, NX=7, ax1=(1, 3, 2), ax2=(0, 5, 4), r=3.0, L=2.0, xi_in=-2.0, xi_out=5.0),
    dict(NL=10, NX=6, ax1=(1, 5, 4), ax2=(0, 6, 4), r=1.5, Kn=0.5),
])
def test_rest_state_is_stationary(kw):
    """n = 1, u = 0, T = 1 with walls at rest and equal reservoirs: advection through the
    curved grid is cancelled exactly by the connection terms."""
    o = ChannelOracle(n_in=1.0, n_out=1.0, **kw)
    F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    L, flux, nw = o.L(F)
    assert np.abs(L).max() <= 1e-13 * np.abs(F).max()
    assert np.allclose(nw, 1.0, rtol=0, atol=1e-13)
    assert np.abs(flux).max() <= 1e-14


@pytest.mark.parametrize("seed", [1, 2])
def test_particle_balance_against_end_fluxes(seed):
    """For any state, d/dt sum_cells dchi dlambda sum_k f' equals the inlet flux minus
    the outlet flux: the walls pass no particles (n_w), the flux differences telescope
    and the force and collision terms conserve particle number."""
    o = ChannelOracle(NL=8, NX=9, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.2, n_in=1.1, n_out=0.9)
    F = _perturbed(o, seed)
    L, flux, _ = o.L(F)
    dN = float((o.vol * L[0].sum(-1)).sum())
    assert dN == pytest.approx(flux[0] - flux[-1], rel=1e-11, abs=1e-14)
    assert abs(flux[0] - flux[-1]) > 1e-3          # the case is not trivially balanced


def test_mirror_symmetry_across_the_centreline():
    """A state symmetric under (lambda, p^lambda) -> (-lambda, -p^lambda) stays symmetric."""
    o = ChannelOracle(NL=8, NX=7, ax1=(1, 4, 3), ax2=(0, 4, 3), Kn=0.1, n_in=1.05, n_out=0.95)
    Qh = o.a1.Q
    mirror_i = np.array([(i + Qh) % (2 * Qh) for i in range(2 * Qh)])
    assert np.allclose(o.a1.p[mirror_i], -o.a1.p, rtol=0, atol=1e-15)

    def M(F):
        G = F.reshape(2, o.NX, o.NL, o.Q1, o.Q2)[:, :, ::-1, mirror_i, :]
        return G.reshape(2, o.NX, o.NL, o.NV)

    F = _perturbed(o, 3)
    F = 0.5 * (F + M(F))
    L, _, nw = o.L(F)
    assert np.abs(L - M(L)).max() <= 1e-13 * np.abs(L).max()
    assert np.allclose(nw[:, 0], nw[:, 1], rtol=1e-13)


@pytest.mark.slow
def test_steady_flux_is_the_same_through_every_cross_section():
    """Pressure-driven flow to r < 1e-10: the particle flux through each xi face agrees
    (closed walls), and it runs from the high- to the low-density reservoir."""
    o = ChannelOracle(NL=6, NX=8, ax1=(1, 3, 2), ax2=(0, 4, 3), Kn=0.3, r=1.5, n_in=1.05, n_out=0.95)
    dt = o.cfl_dt(0.5)
    F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    r = 1.0
    for _ in range(200):
        Fm = o.step(F, dt, 99)
        F = o.step(Fm, dt, 1)
        r = o.residual(F, Fm, dt)
        if r < 1e-10:
            break
    assert r < 1e-10
    _, flux, _ = o.L(F)
    assert flux.min() > 0
    # at r < 1e-10 the mass between two faces still changes by ~ r |F|, about 1e-9 here
    assert (flux.max() - flux.min()) <= 1e-6 * flux.max()


# ---------------------------------------------------------------- the paper's own boundary conditions
def _mirror(o, F):
    """(lambda, p^lambda) -> (-lambda, -p^lambda) of a full-width state."""
    Qh = o.a1.Q
    mi = np.array([(i + Qh) % (2 * Qh) for i in range(2 * Qh)])
    G = F.reshape(2, o.NX, o.NL, o.Q1, o.Q2)[:, :, ::-1, mi, :]
    return G.reshape(2, o.NX, o.NL, o.NV)


@pytest.mark.parametrize("ends,Q0", [(0, 0.0), (1, 0.08)])
def test_half_channel_is_the_upper_half_of_the_full_channel(ends, Q0):
    """Specular centreline (Sec. VI.C.3): for a mirror-symmetric full-width state the
    half channel's L equals the upper half of the full channel's L (the ghost cells hold
    exactly the values the full channel has there)."""
    kw = dict(NX=7, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.1, r=1.8, n_in=1.05, n_out=0.95, ends=ends, Q0=Q0)
    full = ChannelOracle(NL=8, **kw)
    half = ChannelOracle(NL=4, half=True, **kw)
    assert np.array_equal(half.lam_f, full.lam_f[4:])
    F = _perturbed(full, 4)
    F = 0.5 * (F + _mirror(full, F))
    Lf, _, _ = full.L(F)
    Lh, _, nwh = half.L(np.ascontiguousarray(F[:, :, 4:]))
    assert np.abs(Lh - Lf[:, :, 4:]).max() <= 1e-14 * np.abs(Lf).max()
    assert np.all(nwh[:, 0] == 0.0)


@pytest.mark.parametrize("seed", [1, 2])
def test_flow_rate_ends_impose_the_profile(seed):
    """Sec. VI.C.1-2: with the entering populations at f_eq(n_s, u_s, T_w) and n_s from the
    row balance, every lambda row carries exactly the prescribed flow rate through both end
    faces, whatever the state inside."""
    o = ChannelOracle(NL=8, NX=9, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.2, ends=1, Q0=0.1)
    F = _perturbed(o, seed)
    rf = o.end_flow(F)
    assert np.abs(rf[0] - o.profile(0)).max() <= 1e-13
    assert np.abs(rf[1] - o.profile(o.NX)).max() <= 1e-13
    # (1 + phi) Q(lambda) does not depend on phi: the same flux enters and leaves, so the
    # particle content is constant for any state (walls pass nothing, force and collision
    # conserve particles)
    L, flux, _ = o.L(F)
    dN = float((o.vol * L[0].sum(-1)).sum())
    assert abs(flux[0] - flux[-1]) <= 1e-14
    assert abs(dN) <= 1e-12 * abs(flux[0])
    assert flux[0] > 0.05


def test_half_channel_particle_balance():
    """Half channel with reservoir ends: the centreline passes no particles either."""
    o = ChannelOracle(NL=5, NX=8, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.2, half=True, n_in=1.1, n_out=0.9)
    F = _perturbed(o, 3)
    L, flux, _ = o.L(F)
    dN = float((o.vol * L[0].sum(-1)).sum())
    assert dN == pytest.approx(flux[0] - flux[-1], rel=1e-11, abs=1e-14)
