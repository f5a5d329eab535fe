"""GPU parity of the Cartesian-split channel (Sec. VI.G) against the oracle of
``oracle/clb.py``, through the C ABI (FP64; bar 1e-12 relative per distribution)."""
import sys

import numpy as np
import pytest

from oracle.clb import ClbOracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(**kw):
    from paper_1708_05944_amd import ChannelDesc
    o = ClbOracle(NL=kw.pop("N_lambda"), NX=kw.pop("N_xi"), **kw)
    return o, ChannelDesc(N_lambda=o.NL, N_xi=o.NX, cartesian=True, **kw)


def _perturbed(o, seed, amp=0.15):
    rng = np.random.default_rng(seed)
    X, S = np.meshgrid(o.xi_c, o.lam_c, indexing="ij")
    F = o.equilibrium(1 + 0.1 * np.sin(X) * np.cos(2 * S), 0.05 * np.sin(3 * S), 0.2 * np.cos(S) * (1 - S ** 2),
                      1 + 0.05 * np.cos(X + S))
    return F * rng.uniform(1 - amp, 1 + amp, F.shape)


def _relerr(a, b):
    a = np.asarray(a).reshape(2, -1)
    b = np.asarray(b).reshape(2, -1)
    return max(np.abs(a[d] - b[d]).max() / np.abs(b[d]).max() for d in range(2))


CASES = [
    dict(N_lambda=8, N_xi=9, ax1=(1, 4, 3), ax2=(1, 4, 3), Kn=0.1, r=2.5, L=2.0, xi_in=-1.0, xi_out=3.0),   # HH x HH
    dict(N_lambda=7, N_xi=6, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.2, r=1.0),                                 # straight
    dict(N_lambda=6, N_xi=8, ax1=(1, 6, 4), ax2=(1, 6, 4), Kn=0.05, r=2.0, n_in=1.2, n_out=0.9),          # 144 velocities
    dict(N_lambda=9, N_xi=7, ax1=(1, 8, 4), ax2=(1, 8, 4), Kn=0.3, r=3.0, L=2.0, weno_eps=1e-6),          # 256, regularised
    dict(N_lambda=10, N_xi=9, ax1=(1, 4, 3), ax2=(1, 4, 3), Kn=0.1, r=2.5, L=2.0, xi_in=-1.0, xi_out=3.0,
         A=0.95),                                                                                           # stretched
    dict(N_lambda=6, N_xi=9, ax1=(1, 6, 4), ax2=(1, 6, 4), Kn=0.2, r=2.0, L=2.0, xi_in=-1.0, xi_out=3.0,
         half=True, ends=1, Q0=0.1, A=0.95),                                                              # paper's set-up
]


@pytest.mark.parametrize("case", CASES)
def test_clb_operator_matches_oracle(case):
    from paper_1708_05944_amd import Channel
    _say(f"case {case}")
    o, d = _pair(**dict(case))
    c = Channel([d])
    F = _perturbed(o, 5)
    c.set_state(F.ravel())
    L = c.instance_view(c.apply_L(), 0)
    Lw, _ = o.L(F)
    err = _relerr(L, Lw)
    _say(f"L rel err {err:.2e}")
    assert err <= TOL
    c.close()


def test_clb_rest_state_is_stationary():
    from paper_1708_05944_amd import Channel
    o, d = _pair(N_lambda=8, N_xi=9, ax1=(1, 4, 3), ax2=(1, 4, 3), Kn=0.1, r=2.5, L=2.0, xi_in=-1.0, xi_out=3.0,
                 n_in=1.0, n_out=1.0)
    c = Channel([d])
    F0 = c.instance_view(c.get_state(), 0)
    L = c.instance_view(c.apply_L(), 0)
    assert np.abs(L).max() <= 1e-13 * np.abs(F0).max()
    c.close()


def test_clb_and_vielbein_channels_step_together():
    """A batch with two Cartesian-split instances and one vielbein instance: 4 RK3 steps
    of each against its own oracle; the diagnostics of a Cartesian instance take its
    moments as Cartesian components."""
    from oracle.channel import ChannelOracle
    from paper_1708_05944_amd import Channel, ChannelDesc
    o1, d1 = _pair(**dict(CASES[0]))
    o2, d2 = _pair(**dict(CASES[2]))
    kw = dict(ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.1, r=2.0)
    o3 = ChannelOracle(NL=8, NX=9, **kw)
    d3 = ChannelDesc(N_lambda=8, N_xi=9, **kw)
    c = Channel([d1, d3, d2])
    F = [_perturbed(o, 7 + i) for i, o in enumerate((o1, o3, o2))]
    c.set_state(np.concatenate([f.ravel() for f in F]))
    c.step(4)
    G = c.get_state()
    for i, o in enumerate((o1, o3, o2)):
        want = o.step(F[i], c.info[i]["dt"], 4)
        err = _relerr(c.instance_view(G, i), want)
        _say(f"instance {i}: 4 steps rel err {err:.2e}")
        assert err <= TOL
    assert np.isfinite(c.residual()).all()
    got = c.flow_fields(0)
    want = o1.flow_fields(c.instance_view(G, 0))
    m = o1.moments(c.instance_view(G, 0))
    assert np.allclose(got["ux"], m["u1"], rtol=0, atol=1e-15) and np.allclose(got["uy"], m["u2"], rtol=0, atol=1e-15)
    for k in ("P", "psi", "Pw"):
        assert np.abs(got[k] - want[k]).max() <= 1e-12 * np.abs(want[k]).max(), k
    c.close()


def test_clb_paper_setup_steps_match_oracle():
    """The paper's comparison set-up in the Cartesian split: half channel, flow-rate ends,
    stretched lambda -- 4 RK3 steps from a perturbed state."""
    from paper_1708_05944_amd import Channel
    o, d = _pair(**dict(CASES[-1]))
    c = Channel([d])
    F = _perturbed(o, 21)
    c.set_state(F.ravel())
    c.step(4)
    err = _relerr(c.instance_view(c.get_state(), 0), o.step(F, c.info[0]["dt"], 4))
    _say(f"4 steps rel err {err:.2e}")
    assert err <= TOL
    c.close()


def test_vielbein_and_cartesian_split_channels_agree():
    """Sec. VI.G compares the two momentum discretisations on the paper's set-up and finds
    the wall pressure of HH(4;6) x H(4;5) (vielbein) and HH(4;6) x HH(4;6) (Cartesian split)
    overlapped.  Here: half channel with flow-rate ends (Q0 = 0.05), Kn 0.2, 16 x 64 cells
    stretched with A = 0.95, both advanced from rest to t = 8 on the GPU.  Measured on
    MI355X: the upper-wall pressures differ by 0.3 % of their range along the channel and
    u^y by 0.4 % of its maximum (3 % and 2.7 % at t = 1, the start-up transients differing
    most); the bounds are 2.5 times the measured t = 8 values.  This is a property of two
    different velocity-space discretisations of one flow, not parity."""
    import torch
    from paper_1708_05944_amd import Channel, ChannelDesc
    geo = dict(N_lambda=16, N_xi=64, xi_in=-4.0, xi_out=12.0, r=2.0, L=4.0, Kn=0.2, tau_model=1, T_w=1.0, half=True,
               ends=1, Q0=0.05, A=0.95)
    v = Channel([ChannelDesc(ax1=(1, 6, 4), ax2=(0, 5, 4), **geo)])
    c = Channel([ChannelDesc(ax1=(1, 6, 4), ax2=(1, 6, 4), cartesian=True, **geo)])
    for ch in (v, c):
        ch.step(int(round(8.0 / ch.info[0]["dt"])))
    torch.cuda.synchronize()
    fv, fc = v.flow_fields(0), c.flow_fields(0)
    Pv, Pc = fv["Pw"][1], fc["Pw"][1]
    dP = np.abs(Pv - Pc).max() / (Pv.max() - Pv.min())
    du = np.abs(fv["uy"] - fc["uy"]).max() / np.abs(fv["uy"]).max()
    _say(f"wall pressure difference {dP:.2e} of its range, u^y difference {du:.2e} of its max")
    assert dP <= 8e-3 and du <= 1e-2
    v.close()
    c.close()
