"""GPU parity of the expanding-channel path against the FP64 CPU oracle, through the C
ABI.  Bar: max-norm difference per distribution, relative to the oracle's max-norm,
at most 1e-12 (both sides follow the same arithmetic; the GPU fuses multiply-adds)."""
import sys

import numpy as np
import pytest

from oracle.channel import ChannelOracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(**kw):
    from paper_1708_05944_amd import ChannelDesc
    o = ChannelOracle(NL=kw.pop("N_lambda"), NX=kw.pop("N_xi"), **kw)
    d = ChannelDesc(N_lambda=o.NL, N_xi=o.NX, **kw)
    return o, d


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
    dict(N_lambda=8, N_xi=10, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.05),                         # smallest set
    dict(N_lambda=12, N_xi=9, ax1=(1, 8, 4), ax2=(0, 16, 4), Kn=0.05),                        # 256 velocities (config 3)
    dict(N_lambda=7, N_xi=13, ax1=(1, 5, 4), ax2=(0, 7, 4), Kn=0.3, r=3.0, L=2.0),            # p^xi = 0 node, steep
    dict(N_lambda=10, N_xi=6, ax1=(1, 6, 4), ax2=(0, 8, 4), Kn=0.1, r=1.0),                   # straight channel
    dict(N_lambda=6, N_xi=11, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.2, weno_eps=1e-6, n_in=1.2),  # regularised WENO
    dict(N_lambda=7, N_xi=8, ax1=(1, 12, 4), ax2=(0, 8, 4), Kn=0.08),                         # 24 x 8: two p^lambda tiles
    dict(N_lambda=6, N_xi=7, ax1=(1, 4, 3), ax2=(0, 20, 4), Kn=0.15, r=2.5),                  # 8 x 20: two p^xi tiles
    dict(N_lambda=5, N_xi=9, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.1, half=True),                 # specular centreline
    dict(N_lambda=8, N_xi=9, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.2, ends=1, Q0=0.1),            # flow-rate ends
    dict(N_lambda=6, N_xi=8, ax1=(1, 8, 4), ax2=(0, 16, 4), Kn=0.05, half=True, ends=1, Q0=0.08),  # the paper's set-up
    dict(N_lambda=10, N_xi=9, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=0.1, r=2.0, L=2.0, xi_in=-1.0, xi_out=3.0,
         A=0.95),                                                                                   # stretched lambda
    dict(N_lambda=6, N_xi=8, ax1=(1, 8, 4), ax2=(0, 16, 4), Kn=0.05, half=True, ends=1, Q0=0.08,
         A=0.95),                                                                                   # paper's set-up and grid
]


@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("case", CASES)
def test_channel_operator_matches_oracle(case, kernel):
    """Both FP64 kernels on every case: the velocity tiles on the matrix cores (1) and the
    population kernel (2)."""
    from paper_1708_05944_amd import Channel
    _say(f"case {case}, kernel {kernel}")
    o, d = _pair(**dict(case))
    d.kernel = kernel
    c = Channel([d])
    F = _perturbed(o, 5)
    c.set_state(F.ravel())
    L = c.instance_view(c.apply_L(), 0)
    Lw, _, _ = o.L(F)
    err = _relerr(L, Lw)
    _say(f"L rel err {err:.2e}")
    assert err <= TOL
    c.close()


def test_channel_initial_state_and_rest_stationarity():
    """The library starts from the rest Maxwellian, which with equal reservoirs is a
    fixed point of the curved-channel scheme to rounding."""
    from paper_1708_05944_amd import Channel
    o, d = _pair(N_lambda=12, N_xi=9, ax1=(1, 8, 4), ax2=(0, 16, 4), Kn=0.05, n_in=1.0, n_out=1.0)
    c = Channel([d])
    F0 = c.instance_view(c.get_state(), 0)
    assert _relerr(F0, o.equilibrium(1.0, 0.0, 0.0, 1.0)) <= 1e-14
    L = c.instance_view(c.apply_L(), 0)
    assert np.abs(L).max() <= 1e-13 * np.abs(F0).max()
    c.close()


def test_channel_steps_match_oracle():
    """20 RK3 steps of the pressure-driven flow from a perturbed state."""
    from paper_1708_05944_amd import Channel
    o, d = _pair(N_lambda=8, N_xi=12, ax1=(1, 4, 3), ax2=(0, 6, 4), Kn=0.1)
    c = Channel([d])
    F = _perturbed(o, 7)
    c.set_state(F.ravel())
    c.step(20)
    want = o.step(F, c.info[0]["dt"], 20)
    err = _relerr(c.instance_view(c.get_state(), 0), want)
    _say(f"20 steps rel err {err:.2e}")
    assert err <= TOL
    r = c.residual()[0]
    Fm = o.step(F, c.info[0]["dt"], 19)
    assert abs(r / o.residual(want, Fm, c.info[0]["dt"]) - 1) <= 1e-9
    c.close()


def test_channel_uneven_batch_matches_oracle():
    from paper_1708_05944_amd import Channel
    # three velocity-tile classes in one batch (one launch per class)
    pairs = [_pair(**dict(CASES[0])), _pair(**dict(CASES[5])), _pair(**dict(CASES[2])), _pair(**dict(CASES[6])),
             _pair(**dict(CASES[1]))]
    c = Channel([p[1] for p in pairs])
    st = c.get_state()
    inits = []
    for i, (o, _) in enumerate(pairs):
        F = _perturbed(o, 20 + i)
        c.instance_view(st, i)[...] = F
        inits.append(F)
    c.set_state(st)
    c.step(5)
    got = c.get_state()
    for i, (o, _) in enumerate(pairs):
        want = o.step(inits[i], c.info[i]["dt"], 5)
        err = _relerr(c.instance_view(got, i), want)
        _say(f"instance {i}: rel err {err:.2e}")
        assert err <= TOL
    c.close()


def test_channel_paper_boundary_conditions_steps_match_oracle():
    """20 RK3 steps of the half channel with flow-rate ends from rest."""
    from paper_1708_05944_amd import Channel
    o, d = _pair(**dict(CASES[9]))
    c = Channel([d])
    F0 = c.instance_view(c.get_state(), 0).copy()
    c.step(20)
    want = o.step(F0, c.info[0]["dt"], 20)
    err = _relerr(c.instance_view(c.get_state(), 0), want)
    _say(f"half channel, flow-rate ends, 20 steps rel err {err:.2e}")
    assert err <= TOL
    c.close()


def test_channel_moments_and_content():
    from paper_1708_05944_amd import Channel
    o, d = _pair(**dict(CASES[2]))
    c = Channel([d])
    F = _perturbed(o, 9)
    c.set_state(F.ravel())
    m = c.moments(0)
    mw = o.moments(F)
    for key in ("n", "u1", "u2", "T"):
        assert np.abs(m[key] - mw[key]).max() <= 1e-12 * max(np.abs(mw[key]).max(), 1e-3), key
    assert m["content"].sum() == pytest.approx(o.mass(F), rel=1e-13)
    c.close()


def test_channel_total_mass_open_bc_and_run_seconds():
    """vlb_channel_total_mass equals the oracle's particle number of the same state;
    vlb_channel_set_open_bc on an instance created with equal reservoirs gives bitwise the
    steps of an instance created with the new reservoir density, in both precisions
    (and, with n = 1 at both ends again, the rest state is stationary again); the run to
    steady state reports its wall-clock seconds.  The batch runs in a torch-allocated
    workspace bound through vlb_channel_bind_workspace."""
    from paper_1708_05944_amd import VLB_MIXED, Channel
    o, d = _pair(N_lambda=10, N_xi=12, ax1=(1, 4, 3), ax2=(0, 6, 4), Kn=0.1, n_in=1.0, n_out=1.0)
    for prec in (0, VLB_MIXED):
        c = Channel([d], precision=prec)
        F = _perturbed(o, 11)
        c.set_state(F.ravel())
        assert c.total_mass()[0] == pytest.approx(o.mass(F), rel=1e-13)
        c.set_state(o.equilibrium(1.0, 0.0, 0.0, 1.0).ravel())
        c.set_open_bc(0, 0, 1.15, 1.0)
        c.set_open_bc(0, 1, 0.9, 1.0)
        c.step(30)
        a = c.get_state()
        _, d2 = _pair(N_lambda=10, N_xi=12, ax1=(1, 4, 3), ax2=(0, 6, 4), Kn=0.1, n_in=1.15, n_out=0.9)
        c2 = Channel([d2], precision=prec)
        c2.set_state(o.equilibrium(1.0, 0.0, 0.0, 1.0).ravel())
        c2.step(30)
        assert np.array_equal(a, c2.get_state()), prec
        c2.close()
        c.set_open_bc(0, 0, 1.0, 1.0)
        c.set_open_bc(0, 1, 1.0, 1.0)
        c.set_state(o.equilibrium(1.0, 0.0, 0.0, 1.0).ravel())
        c.step(5)
        assert c.residual()[0] < 1e-10
        c.close()
    c = Channel([d])
    c.set_open_bc(0, 0, 1.05, 1.0)
    steps, r, ok = c.run_to_steady(1e-3, 20_000, 500)
    _say(f"run to r < 1e-3: {steps[0]} steps in {c.last_run_seconds():.3f} s")
    assert ok and c.last_run_seconds() > 0
    c.close()


def test_channel_init_equilibrium_matches_oracle():
    """vlb_channel_init_equilibrium builds the local equilibrium of given per-cell fields
    (n, u^lambda, u^xi, T) as the oracle's equilibrium does (1e-13 relative), for the
    second instance of an uneven batch in both precisions, leaving the first untouched."""
    from paper_1708_05944_amd import VLB_MIXED, Channel
    o0, d0 = _pair(N_lambda=8, N_xi=6, ax1=(1, 4, 3), ax2=(0, 6, 4), Kn=0.1)
    o, d = _pair(N_lambda=10, N_xi=12, ax1=(1, 8, 4), ax2=(0, 16, 4), Kn=0.05, r=2.5)
    X, S = np.meshgrid(o.xi_c, o.lam_c, indexing="ij")
    fields = (1 + 0.1 * np.sin(X) * np.cos(2 * S), 0.05 * np.sin(3 * S), 0.2 * np.cos(S) * (1 - S ** 2),
              1 + 0.05 * np.cos(X + S))
    want = o.equilibrium(*fields)
    for prec in (0, VLB_MIXED):
        c = Channel([d0, d], precision=prec)
        before = c.get_instance_state(0)
        c.init_equilibrium(1, *fields)
        err = _relerr(c.get_instance_state(1), want)
        _say(f"precision {prec}: init_equilibrium rel err {err:.2e}")
        assert err <= 1e-13
        assert np.array_equal(c.get_instance_state(0), before)
        c.close()


# ---------------------------------------------------------------- mixed precision
# FP32 stage kernel on populations scaled by 1/(w_i w_j), FP64 moment / wall-flux /
# residual sums.  Operator bar: relative max-norm 2e-6 (about 30 ulp of float), against
# the oracle evaluated on the FP32-rounded state the kernel actually reads.
MIXED_CASES = [CASES[1], CASES[0], CASES[4], CASES[5], CASES[6], CASES[7], CASES[8], CASES[9]]


@pytest.mark.parametrize("case", MIXED_CASES)
def test_channel_fp32_operator_matches_oracle(case):
    from paper_1708_05944_amd import VLB_MIXED, Channel
    _say(f"fp32 case {case}")
    o, d = _pair(**dict(case))
    c = Channel([d], precision=VLB_MIXED)
    c.set_state(_perturbed(o, 11).ravel())
    c.step(0)                                   # moves the state into the FP32 buffers
    Fr = c.instance_view(c.get_state(), 0).copy()   # the rounded state, back in FP64
    c.step(0)
    L = c.instance_view(c.apply_L(), 0)
    Lw, _, _ = o.L(Fr)
    err = _relerr(L, Lw)
    _say(f"fp32 L rel err {err:.2e}")
    assert err <= 2e-6
    c.close()


def test_channel_mixed_steady_state_matches_fp64():
    """Pressure-driven flow to r < 1e-10: FP32 phase + FP64 polish against FP64 alone;
    every moment profile within 1e-5 (relative to max(|profile|, 1e-3))."""
    from paper_1708_05944_amd import VLB_MIXED, Channel
    kw = dict(N_lambda=6, N_xi=8, ax1=(1, 3, 2), ax2=(0, 4, 3), Kn=0.3, r=1.5, n_in=1.05, n_out=0.95)
    runs = {}
    for name, prec in (("fp64", 0), ("mixed", VLB_MIXED)):
        o, d = _pair(**dict(kw))
        c = Channel([d], precision=prec)
        steps, r, ok = c.run_to_steady(1e-10, 400_000, 500)
        _say(f"{name}: steps {steps[0]} r {r[0]:.2e} fp32 steps {c.fp32_steps()}")
        assert ok
        runs[name] = c.moments(0)
        if prec:
            assert c.fp32_steps() > 0
        c.close()
    for key in ("n", "u1", "u2", "T"):
        a, b = runs["mixed"][key], runs["fp64"][key]
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-3)
        _say(f"{key}: mixed vs fp64 {err:.2e}")
        assert err <= 1e-5, key


def test_channel_flow_fields_match_oracle():
    """Diagnostics of Sec. VI.D / VI.F (Cartesian velocity, pressure, stream function,
    vorticity, wall pressures) of every instance of a mixed batch -- odd and even N_lambda,
    the half channel, the straight channel, the paper's set-up -- computed on the device
    from seeded perturbed states, against the oracle's; per field, max difference over the
    oracle's max-norm <= 1e-12."""
    from paper_1708_05944_amd import Channel
    picks = [CASES[2], CASES[7], CASES[9], CASES[3]]
    pairs = [_pair(**dict(cs)) for cs in picks]
    c = Channel([d for _, d in pairs])
    states = [_perturbed(o, 11 + i) for i, (o, _) in enumerate(pairs)]
    c.set_state(np.concatenate([F.ravel() for F in states]))
    for i, (o, _) in enumerate(pairs):
        _say(f"flow fields of instance {i}: {picks[i]}")
        got = c.flow_fields(i)
        want = o.flow_fields(states[i])
        for k, w in want.items():
            err = np.abs(got[k] - w).max() / np.abs(w).max()
            _say(f"  {k}: rel err {err:.2e}")
            assert got[k].shape == w.shape and err <= TOL, (k, err)
    c.close()


def test_channel_flow_fields_of_mixed_batch():
    """A mixed-precision batch moves its FP32 state to FP64 and reports the fields of
    that state.  Starting from rest, the cross-stream velocity is still far below the
    streamwise one, so both velocity components are measured on the speed scale."""
    from paper_1708_05944_amd import VLB_MIXED, Channel
    o, d = _pair(**dict(CASES[9]))
    c = Channel([d], precision=VLB_MIXED)
    c.step(20)
    F = c.get_instance_state(0)
    got = c.flow_fields(0)
    want = o.flow_fields(F)
    speed = max(np.abs(want["ux"]).max(), np.abs(want["uy"]).max())
    for k, w in want.items():
        err = np.abs(got[k] - w).max() / (speed if k in ("ux", "uy") else np.abs(w).max())
        _say(f"  {k}: rel err {err:.2e}")
        assert err <= TOL, (k, err)
    assert np.abs(want["psi"]).max() > 0                 # the flow-rate ends drive a flow
    c.close()


def test_channel_step_graphs_are_bitwise_identical():
    """Runs of more than ten steps replay a captured graph of ten steps: 25 steps (two
    replays and five plain steps), twice with host reads in between, match plain launches
    bit for bit -- a batch of two vielbein tile classes and a Cartesian-split instance in
    FP64, and a mixed-precision vielbein batch."""
    from paper_1708_05944_amd import VLB_MIXED, Channel, ChannelDesc
    descs = [ChannelDesc(N_lambda=12, N_xi=9, ax1=(1, 8, 4), ax2=(0, 16, 4), Kn=0.05),
             ChannelDesc(N_lambda=7, N_xi=8, ax1=(1, 12, 4), ax2=(0, 8, 4), Kn=0.08),
             ChannelDesc(N_lambda=8, N_xi=9, ax1=(1, 4, 3), ax2=(1, 4, 3), Kn=0.1, r=2.5, L=2.0, xi_in=-1.0,
                         xi_out=3.0, cartesian=True)]
    for prec, ds in ((0, descs), (VLB_MIXED, descs[:2])):
        a, b = Channel(ds, precision=prec), Channel(ds, precision=prec)
        b.set_graphs(False)
        for rnd in range(2):
            a.step(25)
            b.step(25)
            Fa, Fb = a.get_state(), b.get_state()
            _say(f"precision {prec} round {rnd}: max |diff| {np.abs(Fa - Fb).max():.1e}")
            assert np.array_equal(Fa, Fb)
            assert np.array_equal(a.residual(), b.residual())
        a.close()
        b.close()


def test_population_kernel_takes_sets_beyond_two_tiles():
    """HH(4;24) x H(4;5): 48 x 5 nodes need three 16-node tiles along p^lambda, which the
    tile kernel does not take; the automatic choice runs it on the population kernel
    (FP64) -- operator and three steps against the oracle, in the expansion with the
    paper's half channel, flow-rate ends and stretched lambda."""
    from paper_1708_05944_amd import Channel
    kw = dict(N_lambda=6, N_xi=9, ax1=(1, 24, 4), ax2=(0, 5, 4), Kn=0.2, r=2.0, L=2.0, xi_in=-1.0, xi_out=3.0,
              half=True, ends=1, Q0=0.1, A=0.95)
    o, d = _pair(**dict(kw))
    c = Channel([d])
    F = _perturbed(o, 13)
    c.set_state(F.ravel())
    err = _relerr(c.instance_view(c.apply_L(), 0), o.L(F)[0])
    _say(f"L rel err {err:.2e}")
    assert err <= TOL
    c.set_state(F.ravel())
    c.step(3)
    err = _relerr(c.instance_view(c.get_state(), 0), o.step(F, c.info[0]["dt"], 3))
    _say(f"3 steps rel err {err:.2e}")
    assert err <= TOL
    c.close()
