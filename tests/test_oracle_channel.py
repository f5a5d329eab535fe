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
    dict(NL=10, NX=9, ax1=(1, 4, 3), ax2=(0, 5, 4), r=2.0, L=2.0, xi_in=-1.0, xi_out=3.0, A=0.95),   # stretched
    dict(NL=7, NX=8, ax1=(1, 4, 3), ax2=(0, 5, 4), r=2.5, half=True, A=0.95),                    # paper's grid
])
def test_rest_state_is_stationary(kw):
    """n = 1, u = 0, T = 1 with walls at rest and equal reservoirs: advection through the
    curved grid is cancelled exactly by the connection terms."""
    o = ChannelOracle(n_in=1.0, n_out=1.0, **kw)
    F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    L, flux, nw = o.L(F)
    assert np.abs(L).max() <= 1e-13 * np.abs(F).max()
    walls = nw[:, 1:] if kw.get("half") else nw          # the half channel has its wall at lambda = 1 only
    assert np.allclose(walls, 1.0, rtol=0, atol=1e-13)
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


@pytest.mark.parametrize("ends,Q0,A", [(0, 0.0, 0.0), (1, 0.08, 0.0), (1, 0.08, 0.95)])
def test_half_channel_is_the_upper_half_of_the_full_channel(ends, Q0, A):
    """Specular centreline (Sec. VI.C.3): for a mirror-symmetric full-width state the
    half channel's L equals the upper half of the full channel's L (the ghost cells hold
    exactly the values the full channel has there)."""
    kw = dict(NX=7, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.1, r=1.8, n_in=1.05, n_out=0.95, ends=ends, Q0=Q0, A=A)
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


# ---------------------------------------------------------------- diagnostics (Sec. VI.D, VI.F)
def test_d3_exact_for_quadratics_on_unequal_nodes():
    """The three-point formulas (bulk, first and last node) differentiate any quadratic
    exactly on unequally spaced nodes -- the property they are built on.  A sign slip in
    any weight (the printed last-node formula has one on its first term) fails this."""
    from oracle.channel import d3
    rng = np.random.default_rng(5)
    x = np.sort(rng.uniform(-1, 1, 9))
    a, b, c = rng.normal(size=(3, 4))
    f = a[:, None] + b[:, None] * x[None, :] + c[:, None] * x[None, :] ** 2     # [4][9]
    want = b[:, None] + 2 * c[:, None] * x[None, :]
    assert np.allclose(d3(f, x, 1), want, rtol=0, atol=1e-11)
    assert np.allclose(d3(f.T, x, 0), want.T, rtol=0, atol=1e-11)
    cubic = x ** 3                                                               # and not beyond
    assert np.abs(d3(cubic, x, 0) - 3 * x ** 2).max() > 1e-6


def test_flow_fields_closed_forms():
    """Straight channel (r = 1, phi = 0), n = 1 + 0.1 lambda, u^lambda = 0,
    u^xi = U (1 - lambda^2): u^y = u^xi and u^x = 0; the vorticity d u^y / dx is -2 U lambda
    (the three-point formulas are exact for quadratics); the wall pressures are the linear
    extrapolation of P; psi vanishes on the centreline and steps by -n u^y d lambda."""
    o = ChannelOracle(NL=8, NX=6, ax1=(1, 4, 3), ax2=(0, 6, 4), r=1.0, Kn=0.1)
    U = 0.05
    X, S = np.meshgrid(o.xi_c, o.lam_c, indexing="ij")
    F = o.equilibrium(1 + 0.1 * S, 0.0, U * (1 - S ** 2), 1.0)
    f = o.flow_fields(F)
    m = o.moments(F)
    assert np.abs(f["ux"]).max() <= 1e-15 and np.allclose(f["uy"], m["u2"], rtol=0, atol=1e-15)
    assert np.allclose(f["omega"], -2 * U * S, rtol=0, atol=1e-12)
    P = f["P"]
    for side, (e, i1, i2) in enumerate(((0, 0, 1), (o.NL, o.NL - 1, o.NL - 2))):
        slope = (P[:, i1] - P[:, i2]) / (o.lam_c[i1] - o.lam_c[i2])
        assert np.allclose(f["Pw"][side], P[:, i1] + slope * (o.lam_f[e] - o.lam_c[i1]), rtol=0, atol=1e-14)
    assert abs(f["Pw"][1].mean() - 1.1) < 2e-3 and abs(f["Pw"][0].mean() - 0.9) < 2e-3   # P = n T, T ~ 1
    assert np.abs(f["psi"][:, o.NL // 2]).max() <= 1e-16
    assert np.allclose(np.diff(f["psi"], axis=1), -(m["n"] * f["uy"]) * o.dlam[None, :], rtol=0, atol=1e-16)


def _solenoidal_state(o, U=0.05):
    """Unit density and the Cartesian velocity of the stream function
    psi = -U (lambda - lambda^3 / 3), lambda = x / (1 + phi(y)): the walls are streamlines
    and the flow through every cross-section is the same; written in the cell triads."""
    X, S = np.meshgrid(o.xi_c, o.lam_c, indexing="ij")
    ph = o.phi_c[:, None]
    dph = o.dphi_c[:, None]
    uy = U * (1 - S ** 2) / (1 + ph)
    ux = U * S * dph * (1 - S ** 2) / (1 + ph)
    a = S * dph
    c = 1 / np.sqrt(1 + a * a)
    return o.equilibrium(np.ones_like(S), c * (ux - a * uy), c * (uy + a * ux), 1.0)


def test_stream_function_counts_flow_through_the_expansion():
    """For the solenoidal field the flow -(psi_wall - psi_centre) through every column is
    the midpoint sum of U (1 - lambda^2) over [0, 1], U (2/3 + h^2/12), whatever phi(xi):
    this fixes the width element (1 + phi) d lambda of the column integral."""
    o = ChannelOracle(NL=10, NX=12, ax1=(1, 4, 3), ax2=(0, 6, 4), r=2.0, L=4.0, xi_in=-1.0, xi_out=5.0)
    U, h = 0.05, 0.2
    f = o.flow_fields(_solenoidal_state(o, U))
    want = U * (2 / 3 + h * h / 12)
    assert np.allclose(f["psi"][:, -1], -want, rtol=1e-13, atol=0)
    assert np.allclose(f["psi"][:, 0], want, rtol=1e-13, atol=0)
    assert np.abs(np.diff(o.phi_c)).max() > 0.1        # the columns really differ in width


def test_vorticity_converges_to_curl_at_second_order():
    """Eq. canalie_vorti on the grid against omega = d_x u_y - d_y u_x of the solenoidal
    field, differentiated in Cartesian coordinates (fine central differences of the closed
    form): the error falls by about 4 when both spacings halve."""
    from oracle.channel import wall_phi
    U, r, L = 0.05, 2.0, 4.0

    def cart(x, y):
        ph = wall_phi(y, r, L)
        lam = x / (1 + ph)
        dph = wall_phi(y, r, L, 1)
        return U * lam * dph * (1 - lam ** 2) / (1 + ph), U * (1 - lam ** 2) / (1 + ph)

    errs = []
    for NL, NX in ((16, 24), (32, 48)):
        o = ChannelOracle(NL=NL, NX=NX, ax1=(1, 4, 3), ax2=(0, 6, 4), r=r, L=L, xi_in=-1.0, xi_out=5.0)
        f = o.flow_fields(_solenoidal_state(o, U))
        e = 1e-5
        want = np.empty((NX, NL))
        for p in range(NX):
            for s in range(NL):
                y = o.xi_c[p]
                x = o.lam_c[s] * (1 + o.phi_c[p])
                want[p, s] = ((cart(x + e, y)[1] - cart(x - e, y)[1]) - (cart(x, y + e)[0] - cart(x, y - e)[0])) / (2 * e)
        errs.append(np.abs(f["omega"] - want).max())
    assert errs[0] / errs[1] > 3.2, errs
    assert errs[1] < 2e-3 * U, errs


def test_flow_fields_rotation_keeps_speed():
    """The triad-to-Cartesian rotation of Eq. canalie_u preserves |u| in the expansion."""
    o = ChannelOracle(NL=8, NX=9, ax1=(1, 4, 3), ax2=(0, 5, 4), r=2.5, xi_in=-1.0, xi_out=3.0)
    F = _perturbed(o, 6)
    f = o.flow_fields(F)
    m = o.moments(F)
    assert np.allclose(f["ux"] ** 2 + f["uy"] ** 2, m["u1"] ** 2 + m["u2"] ** 2, rtol=1e-13, atol=1e-18)
    assert np.abs(o.dphi_c).max() > 0.1          # the triad is really tilted here


def test_stretched_lambda_faces():
    """Eq. canalie_stretch with H / 2 = 1: faces tanh(eta) / A on equal eta cells, the walls
    at lambda = +-1 and the cells refined towards them; a mirror-symmetric state keeps its
    symmetry on the stretched grid."""
    o = ChannelOracle(NL=10, NX=7, ax1=(1, 4, 3), ax2=(0, 5, 4), r=2.0, Kn=0.1, A=0.95)
    eta = np.linspace(-np.arctanh(0.95), np.arctanh(0.95), 11)
    assert np.allclose(o.lam_f, np.tanh(eta) / 0.95, rtol=0, atol=1e-15)
    assert o.lam_f[0] == -1.0 and o.lam_f[-1] == 1.0 and o.lam_f[5] == 0.0
    assert o.dlam[0] < 0.2 * o.dlam[4]
    F = _perturbed(o, 9)
    F = 0.5 * (F + _mirror(o, F))
    L, _, _ = o.L(F)
    assert np.abs(L - _mirror(o, L)).max() <= 1e-13 * np.abs(L).max()
