"""Pins of the Cartesian-split channel oracle (Sec. VI.G) in ``oracle/clb.py``: the
uniform rest state is an exact discrete solution in the expansion (free-stream
preservation of the discrete metric), a straight channel reduces it to the vielbein
channel of the independent C oracle (the triad is Cartesian and the forces vanish when
phi = 0), the walls pass no particles (Eq. canalie_coord_nw), and a mirror-symmetric state
keeps its symmetry."""
import numpy as np

from oracle.channel import ChannelOracle
from oracle.clb import ClbOracle


def _perturbed(o, seed, amp=0.15):
    rng = np.random.default_rng(seed)
    X, S = np.meshgrid(o.xi_c, o.lam_c, indexing="ij")
    F = o.equilibrium(1 + 0.1 * np.sin(X) * np.cos(2 * S), 0.05 * np.sin(3 * S), 0.2 * np.cos(S) * (1 - S ** 2),
                      1 + 0.05 * np.cos(X + S))
    return F * rng.uniform(1 - amp, 1 + amp, F.shape)


def test_rest_state_is_stationary_in_the_expansion():
    o = ClbOracle(NL=8, NX=9, ax1=(1, 4, 3), ax2=(1, 3, 2), r=2.0, L=2.0, xi_in=-1.0, xi_out=3.0, Kn=0.1,
                  n_in=1.0, n_out=1.0)
    # the discrete metric is phi' to second order in the xi spacing
    o2 = ClbOracle(NL=8, NX=18, ax1=(1, 4, 3), ax2=(1, 3, 2), r=2.0, L=2.0, xi_in=-1.0, xi_out=3.0, Kn=0.1)
    e1, e2 = np.abs(o.metric - o.dphi_c).max(), np.abs(o2.metric - o2.dphi_c).max()
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)
    F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    L, nw = o.L(F)
    assert np.abs(L).max() <= 1e-13 * np.abs(F).max()
    assert np.abs(nw - 1.0).max() <= 1e-14


def test_straight_channel_is_the_vielbein_channel():
    kw = dict(NL=7, NX=6, ax1=(1, 4, 3), ax2=(0, 5, 4), r=1.0, Kn=0.2, n_in=1.1, n_out=0.9)
    c, v = ClbOracle(**kw), ChannelOracle(**kw)
    F = _perturbed(v, 1)
    Lc, _ = c.L(F)
    Lv, _, _ = v.L(F)
    assert np.abs(Lc - Lv).max() <= 1e-13 * np.abs(Lv).max()


def test_walls_pass_no_particles():
    o = ClbOracle(NL=8, NX=7, ax1=(1, 4, 3), ax2=(1, 3, 2), r=2.5, L=2.0, xi_in=-1.0, xi_out=3.0, Kn=0.1)
    F = _perturbed(o, 2)
    assert np.abs(o.wall_flux(F)).max() <= 1e-15 * np.abs(F[0]).sum(-1).max()
    assert np.abs(o.metric).max() > 0.3                     # populations change side along the wall


def test_mirror_symmetric_state_stays_symmetric():
    o = ClbOracle(NL=8, NX=7, ax1=(1, 4, 3), ax2=(1, 3, 2), r=2.5, L=2.0, xi_in=-1.0, xi_out=3.0, Kn=0.1)
    F = _perturbed(o, 3).reshape(2, o.NX, o.NL, o.Q1, o.Q2)
    Q = o.a1.Q
    perm = np.r_[Q:2 * Q, 0:Q]                              # p^x -> -p^x on the half-range axis
    mirror = lambda G: G[:, :, ::-1][:, :, :, perm, :]
    Fs = 0.5 * (F + mirror(F))
    L = o.L(Fs.reshape(2, o.NX, o.NL, -1))[0].reshape(Fs.shape)
    assert np.abs(L - mirror(L)).max() <= 1e-13 * np.abs(L).max()


def test_rest_state_is_stationary_on_the_stretched_grid():
    o = ClbOracle(NL=10, NX=9, ax1=(1, 4, 3), ax2=(1, 3, 2), r=2.0, L=2.0, xi_in=-1.0, xi_out=3.0, Kn=0.1,
                  n_in=1.0, n_out=1.0, A=0.95)
    F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    L, nw = o.L(F)
    assert np.abs(L).max() <= 1e-13 * np.abs(F).max()


def test_straight_half_channel_with_flow_rate_ends_is_the_vielbein_channel():
    """With phi = 0 the Cartesian split and the vielbein channel coincide also for the
    paper's set-up: specular centreline and flow-rate ends (against the C oracle)."""
    kw = dict(NL=5, NX=6, ax1=(1, 4, 3), ax2=(0, 5, 4), r=1.0, Kn=0.2, half=True, ends=1, Q0=0.08)
    c, v = ClbOracle(**kw), ChannelOracle(**kw)
    F = _perturbed(v, 1)
    Lc, Lv = c.L(F)[0], v.L(F)[0]
    assert np.abs(Lc - Lv).max() <= 1e-13 * np.abs(Lv).max()


def test_flow_rate_ends_impose_the_profile():
    o = ClbOracle(NL=6, NX=7, ax1=(1, 4, 3), ax2=(1, 3, 2), r=2.5, L=2.0, xi_in=-1.0, xi_out=3.0, Kn=0.1, half=True,
                  ends=1, Q0=0.1, A=0.9)
    rf = o.end_flow(_perturbed(o, 2))
    assert np.abs(rf[0] - o.profile(0)).max() <= 1e-14
    assert np.abs(rf[1] - o.profile(o.NX)).max() <= 1e-14


def test_half_channel_is_the_upper_half_of_the_full_channel():
    kw = dict(NX=7, ax1=(1, 4, 3), ax2=(1, 3, 2), r=2.5, L=2.0, xi_in=-1.0, xi_out=3.0, Kn=0.1, ends=1, Q0=0.1, A=0.9)
    full, half = ClbOracle(NL=8, **kw), ClbOracle(NL=4, half=True, **kw)
    F = _perturbed(full, 3).reshape(2, full.NX, full.NL, full.Q1, full.Q2)
    Q = full.a1.Q
    perm = np.r_[Q:2 * Q, 0:Q]
    F = (0.5 * (F + F[:, :, ::-1][:, :, :, perm, :])).reshape(2, full.NX, full.NL, -1)
    Lf = full.L(F)[0]
    Lh = half.L(np.ascontiguousarray(F[:, :, 4:]))[0]
    assert np.abs(Lh - Lf[:, :, 4:]).max() <= 1e-14 * np.abs(Lf).max()
