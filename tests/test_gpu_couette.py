"""GPU parity of the FP64 Couette hot path against the CPU oracle, through the C ABI.

Bar: max-norm difference per distribution, relative to the oracle's max-norm, at most
1e-12 (the FP64 agreement the scheme admits: both sides round differently, e.g. fused
multiply-adds on the GPU, but follow the same arithmetic).
"""
import math
import sys

import numpy as np
import pytest

from oracle.couette import TAU_HYDRO, CouetteOracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(**kw):
    """Oracle and library descriptor of one instance; dt = 0 lets the library pick its
    stable step (advection CFL 0.5, force and relaxation limits), which the test then
    hands to the oracle."""
    from paper_1708_05944_amd import CouetteDesc
    ora = CouetteOracle(**kw)
    return ora, CouetteDesc(**kw)


def _perturbed(o, seed):
    rng = np.random.default_rng(seed)
    R = o.Rc
    F = o.equilibrium(1 + 0.1 * np.sin(3 * R), 0.05 * np.cos(2 * R), 0.2 * np.sin(R), 1 + 0.1 * np.cos(R))
    return F * rng.uniform(0.8, 1.2, F.shape)


def _relerr(a, b):
    a = np.asarray(a).reshape(2, -1)
    b = np.asarray(b).reshape(2, -1)
    return max(np.abs(a[d] - b[d]).max() / np.abs(b[d]).max() for d in range(2))


L_CASES = [
    dict(N_R=64, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1, u_in=0.1),                       # single-instance workload
    dict(N_R=37, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1, u_in=0.3, A=0.95),               # ragged tiles, stretched
    dict(N_R=3, ax1=(1, 4, 3), ax2=(0, 5, 4), Kn=1.0, u_in=0.2, u_out=-0.1, T_out=1.1),  # minimum grid
    dict(N_R=40, ax1=(0, 5, 4), ax2=(0, 5, 4), Kn=1e-3, tau_model=TAU_HYDRO, u_in=0.5),  # p^R = 0 node
    dict(N_R=70, ax1=(1, 8, 4), ax2=(1, 4, 3), Kn=2.0, u_in=0.4, A=0.5, delta=0.3),     # HH x HH
    dict(N_R=50, ax1=(1, 16, 4), ax2=(0, 20, 4), Kn=10.0, u_in=0.5, R_out=3.0),          # 640 velocities (VPT 10)
    dict(N_R=33, ax1=(1, 10, 4), ax2=(0, 9, 4), Kn=0.3, u_in=0.25),                     # 180 velocities (VPT 3)
]


@pytest.mark.parametrize("case", L_CASES)
def test_operator_matches_oracle(case):
    """One application of L[F] (walls, WENO, force, BGK) on a perturbed state."""
    from paper_1708_05944_amd import Batch
    _say(f"case {case}")
    ora, desc = _pair(**dict(case))
    b = Batch([desc])
    F = _perturbed(ora, 3)
    b.set_state(F.ravel())
    L = b.instance_view(b.apply_L(), 0)
    Lw, _ = ora.L(F)
    assert _relerr(L, Lw) <= TOL
    b.close()


def test_rk3_steps_match_oracle():
    """1000 RK3 steps of the single-instance workload from rest."""
    from paper_1708_05944_amd import Batch
    ora, desc = _pair(N_R=64, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1, u_in=0.1)
    b = Batch([desc])
    dt = b.info[0]["dt"]
    F0 = b.instance_view(b.get_state(), 0).copy()
    assert _relerr(F0, ora.equilibrium(1, 0, 0, 1)) <= 1e-14
    b.step(1000)
    got = b.instance_view(b.get_state(), 0)
    want = ora.step(F0, dt, 1000)
    assert _relerr(got, want) <= TOL
    # residual of the last step and the moments agree too
    Fm = ora.step(F0, dt, 999)
    r_want = ora.residual(want, Fm, dt)
    assert abs(b.residual()[0] / r_want - 1) <= 1e-9
    m = b.moments(0)
    mw = ora.moments(want)
    for key in ("n", "u1", "u2", "T", "T12", "q1", "q2"):
        # u^R, q and T^{R phi} are small differences of O(0.1-1) quadrature sums, so the
        # bar is relative to max(|value|, 1e-3)
        scale = max(np.abs(mw[key]).max(), 1e-3)
        assert np.abs(m[key] - mw[key]).max() <= 1e-11 * scale, key
    b.close()


def test_uneven_batch_matches_oracle():
    """Instances of different grids and velocity sets advanced in the same launches."""
    from paper_1708_05944_amd import Batch
    cases = [L_CASES[0], L_CASES[1], L_CASES[4], L_CASES[5], L_CASES[6],
             dict(N_R=129, ax1=(1, 6, 4), ax2=(0, 7, 4), Kn=0.05, u_in=0.2, R_out=1.5)]
    pairs = [_pair(**dict(c)) for c in cases]
    b = Batch([p[1] for p in pairs])
    st = b.get_state()
    inits = []
    for i, (ora, _) in enumerate(pairs):
        F = _perturbed(ora, 10 + i)
        b.instance_view(st, i)[...] = F
        inits.append(F)
    b.set_state(st)
    b.step(30)
    got = b.get_state()
    for i, (ora, _) in enumerate(pairs):
        _say(f"instance {i}: {cases[i]}")
        want = ora.step(inits[i], b.info[i]["dt"], 30)
        assert _relerr(b.instance_view(got, i), want) <= TOL, i
    b.close()


def test_particle_number_conserved_on_gpu():
    from paper_1708_05944_amd import Batch
    ora, desc = _pair(N_R=64, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1, u_in=0.1)
    b = Batch([desc])
    m0 = b.total_mass()[0]
    assert abs(m0 / ora.mass(ora.equilibrium(1, 0, 0, 1)) - 1) <= 1e-14
    b.step(10000)
    assert abs(b.total_mass()[0] / m0 - 1) <= 1e4 * 2.2e-16
    b.close()


def test_steady_state_matches_oracle():
    """Single-instance workload to r < 1e-10: the GPU takes exactly the oracle's step
    count and lands on the same state; its own residual is below 1e-10 there."""
    from paper_1708_05944_amd import Batch
    ora, desc = _pair(N_R=64, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1, u_in=0.1)
    b = Batch([desc])
    dt = b.info[0]["dt"]
    F = ora.equilibrium(1, 0, 0, 1)
    steps = 0
    while True:
        F = ora.step(F, dt, 499)
        Fn = ora.step(F, dt, 1)
        steps += 500
        r = ora.residual(Fn, F, dt)
        F = Fn
        if r < 1e-10 or steps > 60000:
            break
    assert r < 1e-10
    b.step(steps)
    assert b.residual()[0] < 1e-10
    assert _relerr(b.instance_view(b.get_state(), 0), F) <= TOL
    b.close()


def test_run_to_steady_and_errors():
    from paper_1708_05944_amd import Batch, VlbError
    ora, desc = _pair(N_R=32, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1, u_in=0.1)
    b = Batch([desc])
    with pytest.raises(VlbError) as e:
        b.residual()
    assert e.value.status == -4
    bad = b.get_state()
    bad[5] = math.nan
    with pytest.raises(VlbError) as e:
        b.set_state(bad)
    assert e.value.status == -6
    steps, r, ok = b.run_to_steady(1e-10, 40000, 500)
    assert ok and r[0] < 1e-10 and steps[0] > 0
    b.close()


def test_unstable_dt_is_rejected():
    """An explicit dt beyond the force-operator limit of the RK3 stability region is
    refused with VLB_EUNSTABLE (HH(4;16) x H(4;20): rho(force) ~ 1.8e3)."""
    from paper_1708_05944_amd import Batch, CouetteDesc, VlbError
    with pytest.raises(VlbError) as e:
        Batch([CouetteDesc(N_R=50, ax1=(1, 16, 4), ax2=(0, 20, 4), Kn=10.0, u_in=0.5, R_out=3.0, dt=2e-3)])
    assert e.value.status == -7


def test_step_graph_replay_is_bitwise_identical():
    """Steps replayed from the captured HIP graph equal plain launches bit for bit, for
    several replays with host work and synchronisation in between, in both precisions."""
    from paper_1708_05944_amd import VLB_MIXED, Batch
    cases = [L_CASES[0], L_CASES[5], L_CASES[6]]
    for prec in (0, VLB_MIXED):
        runs = []
        for graphs in (True, False):
            b = Batch([_pair(**dict(c))[1] for c in cases], precision=prec)
            b.set_persistent(0)
            b.set_graphs(graphs)
            states = []
            for rep in range(3):
                b.step(25)                  # two graph replays + 5 plain steps per call
                states.append(b.get_state())
            runs.append((states, b.residual()))
            b.close()
        for a, c in zip(runs[0][0], runs[1][0]):
            assert np.array_equal(a, c), prec
        assert np.array_equal(runs[0][1], runs[1][1])


def test_multi_step_launch_is_bitwise_identical():
    """Multi-step cooperative launches (grid barrier between stages) equal plain
    launches bit for bit: an uneven small batch stepped in both precisions over several
    calls, and the single-instance workload run to r < 1e-10 in FP64 and by the defect
    correction (whose linearised FP32 steps also take them): same step counts, residuals
    and states."""
    from paper_1708_05944_amd import VLB_MIXED, Batch, workloads
    cases = [L_CASES[0], L_CASES[5], L_CASES[6]]
    for prec in (0, VLB_MIXED):
        runs = []
        for multi in (True, False):
            b = Batch([_pair(**dict(c))[1] for c in cases], precision=prec)
            b.set_persistent(64 if multi else 0)
            if not multi:
                b.set_graphs(False)
            states = []
            for rep in range(3):
                b.step(25 + rep)
                states.append(b.get_state())
            runs.append((states, b.residual()))
            b.close()
        for a, c in zip(runs[0][0], runs[1][0]):
            assert np.array_equal(a, c), prec
        assert np.array_equal(runs[0][1], runs[1][1])
    for prec in (0, VLB_MIXED):
        out = []
        for multi in (True, False):
            b = Batch([workloads.single_couette()], precision=prec)
            b.set_persistent(64 if multi else 0)
            steps, r, ok = b.run_to_steady(1e-10, 40_000, 500)
            assert b.last_run_seconds() > 0
            out.append((steps, r, b.get_state()))
            b.close()
        _say(f"precision {prec}: steps {out[0][0]} / {out[1][0]}, r {out[0][1]} / {out[1][1]}")
        assert out[0][0][0] > 0 and np.array_equal(out[0][0], out[1][0])
        assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def test_single_instance_step_time_is_stated():
    """Time per RK3 step of the single-instance workload (64 cells, 32 velocities, FP64)
    with multi-step launches against graph-replayed and plain launches (reported, with a
    loose sanity bound: all three are bound by the stage kernel's latency, about 16 us per
    stage, not by launches)."""
    import time

    import torch

    from paper_1708_05944_amd import Batch, workloads
    res = {}
    for mode in ("multi", "graphs", "plain"):
        b = Batch([workloads.single_couette()])
        b.autotune(20)
        b.set_persistent(64 if mode == "multi" else 0)
        if mode == "plain":
            b.set_graphs(False)
        b.step(200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(4000)
        torch.cuda.synchronize()
        res[mode] = (time.perf_counter() - t0) / 4000 * 1e6
        b.close()
    _say("us per step: " + ", ".join(f"{k} {v:.1f}" for k, v in res.items()))
    assert all(v < 200 for v in res.values())


@pytest.mark.parametrize("tile", [1, 2, 5, 32])
def test_tile_choice_does_not_change_results(tile):
    """Every cells-per-run choice gives the oracle's result (uneven batch, 20 steps)."""
    from paper_1708_05944_amd import Batch
    cases = [L_CASES[0], L_CASES[2], L_CASES[5], L_CASES[6]]
    pairs = [_pair(**dict(c)) for c in cases]
    b = Batch([p[1] for p in pairs])
    b.set_tile(tile)
    st = b.get_state()
    inits = []
    for i, (ora, _) in enumerate(pairs):
        F = _perturbed(ora, 20 + i)
        b.instance_view(st, i)[...] = F
        inits.append(F)
    b.set_state(st)
    b.step(20)
    got = b.get_state()
    for i, (ora, _) in enumerate(pairs):
        want = ora.step(inits[i], b.info[i]["dt"], 20)
        assert _relerr(b.instance_view(got, i), want) <= TOL, (tile, i)
    b.close()


def test_autotune_keeps_state_and_picks_a_tile():
    from paper_1708_05944_amd import Batch
    b = Batch([_pair(**dict(L_CASES[0]))[1], _pair(**dict(L_CASES[5]))[1]])
    b.step(3)
    before = b.get_state()
    tile, ms = b.autotune(3)
    assert 1 <= tile <= 32 and ms > 0 and b.tile() == tile
    assert np.array_equal(b.get_state(), before)
    b.close()


REG_CASE = dict(N_R=45, ax1=(1, 11, 4), ax2=(0, 13, 4), Kn=0.45, u_in=0.43, R_out=1.42)


@pytest.mark.parametrize("eps", [1e-6, 1.0])
def test_regularised_weno_matches_oracle(eps):
    """The optional regularised WENO weights (weno_eps > 0): operator and 20 steps."""
    from paper_1708_05944_amd import Batch
    ora, desc = _pair(**REG_CASE, weno_eps=eps)
    b = Batch([desc])
    F = _perturbed(ora, 31)
    b.set_state(F.ravel())
    L = b.instance_view(b.apply_L(), 0)
    Lw, _ = ora.L(F)
    assert _relerr(L, Lw) <= TOL
    b.step(20)
    want = ora.step(F, b.info[0]["dt"], 20)
    assert _relerr(b.instance_view(b.get_state(), 0), want) <= TOL
    b.close()


def test_regularisation_lets_a_stalled_instance_converge():
    """HH(4;11) x H(4;13), Kn = 0.45: with the paper's epsilon-free weights the residual
    stalls near 1e-4 (the weights chatter at truncation-error level); with weno_eps =
    1e-6 the same instance reaches r < 1e-10, conserving its particle number."""
    from paper_1708_05944_amd import Batch, CouetteDesc
    d0 = CouetteDesc(N_R=32, ax1=(1, 11, 4), ax2=(0, 13, 4), Kn=0.4454, u_in=0.4349, R_out=1.4182)
    b = Batch([d0])
    b.step(30000)
    r0 = b.residual()[0]
    b.close()
    _say(f"epsilon-free residual after 30000 steps: {r0:.2e}")
    assert r0 > 1e-6
    d0.weno_eps = 1e-6
    b = Batch([d0])
    m0 = b.total_mass()[0]
    steps, r, ok = b.run_to_steady(1e-10, 200000, 500)
    _say(f"regularised: r < 1e-10 after {steps[0]} steps")
    assert ok and r[0] < 1e-10
    assert abs(b.total_mass()[0] / m0 - 1) <= steps[0] * 2.2e-16
    b.close()
