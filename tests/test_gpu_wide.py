"""GPU parity of the large-velocity-set Couette stage (more than 1024 velocities, or
more than 64 nodes on the two axes together) against the FP64 CPU oracle, through the C
ABI.  Bar as for the one-block stage kernel: max-norm difference per distribution over
the oracle's max-norm at most 1e-12."""
import sys

import numpy as np
import pytest

from oracle.couette import CouetteOracle

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(**kw):
    from paper_1708_05944_amd import CouetteDesc
    return CouetteOracle(**kw), CouetteDesc(**kw)


def _perturbed(o, seed):
    rng = np.random.default_rng(seed)
    R = o.Rc
    F = o.equilibrium(1 + 0.1 * np.sin(3 * R), 0.05 * np.cos(2 * R), 0.2 * np.sin(R), 1 + 0.1 * np.cos(R))
    return F * rng.uniform(0.8, 1.2, F.shape)


def _relerr(a, b):
    a = np.asarray(a).reshape(2, -1)
    b = np.asarray(b).reshape(2, -1)
    return max(np.abs(a[d] - b[d]).max() / np.abs(b[d]).max() for d in range(2))


WIDE_CASES = [
    # HH(4;36) x HH(4;10): 1440 velocities, 72 x 20 nodes (ragged 16 x 16 product tiles), stretched
    dict(N_R=8, ax1=(1, 36, 4), ax2=(1, 10, 4), Kn=0.1, u_in=0.5, A=0.5, delta=0.75),
    # 1000 velocities but 40 + 25 nodes: past the one-block kernel's node limit
    dict(N_R=5, ax1=(1, 20, 4), ax2=(0, 25, 4), Kn=1.0, u_in=0.3, u_out=-0.1, T_out=1.1),
    # minimum grid, 36 x 30 nodes
    dict(N_R=3, ax1=(1, 18, 3), ax2=(0, 30, 4), Kn=0.5, u_in=0.2),
]


@pytest.mark.parametrize("case", WIDE_CASES)
def test_wide_operator_matches_oracle(case):
    from paper_1708_05944_amd import Batch
    _say(f"case {case}")
    o, d = _pair(**dict(case))
    b = Batch([d])
    F = _perturbed(o, 7)
    b.set_state(F.ravel())
    L = b.instance_view(b.apply_L(), 0)
    Lw, _ = o.L(F)
    err = _relerr(L, Lw)
    _say(f"L rel err {err:.2e}")
    assert err <= TOL
    b.close()


def test_wide_and_narrow_instances_step_together():
    """A batch holding a one-block instance and two large-set instances: 12 RK3 steps
    (ten through the captured step graph) against the oracle's steps."""
    from paper_1708_05944_amd import Batch
    cases = [dict(N_R=33, ax1=(1, 10, 4), ax2=(0, 9, 4), Kn=0.3, u_in=0.25), WIDE_CASES[0], WIDE_CASES[1]]
    pairs = [_pair(**dict(c)) for c in cases]
    b = Batch([d for _, d in pairs])
    F0 = [_perturbed(o, 11 + i) for i, (o, _) in enumerate(pairs)]
    b.set_state(np.concatenate([F.ravel() for F in F0]))
    b.step(12)
    G = b.get_state()
    for i, (o, _) in enumerate(pairs):
        want = o.step(F0[i], b.info[i]["dt"], 12)
        err = _relerr(b.instance_view(G, i), want)
        _say(f"instance {i} ({cases[i]['ax1']} x {cases[i]['ax2']}): 12 steps rel err {err:.2e}")
        assert err <= TOL
    r = b.residual()
    assert np.isfinite(r).all()
    b.close()


def test_wide_rest_state_is_stationary_and_mass_is_conserved():
    from paper_1708_05944_amd import Batch
    o, d = _pair(N_R=8, ax1=(1, 36, 4), ax2=(1, 10, 4), Kn=0.1, u_in=0.0, A=0.5, delta=0.75)
    b = Batch([d])
    F0 = b.instance_view(b.get_state(), 0)
    L = b.instance_view(b.apply_L(), 0)
    assert np.abs(L).max() <= 1e-13 * np.abs(F0).max()
    o2, d2 = _pair(**dict(WIDE_CASES[0]))
    b2 = Batch([d2])
    b2.set_state(_perturbed(o2, 5).ravel())
    m0 = b2.total_mass()[0]
    b2.step(40)
    m1 = b2.total_mass()[0]
    _say(f"mass {m0!r} -> {m1!r}")
    assert abs(m1 - m0) <= 1e-13 * m0
    b.close()
    b2.close()


def test_wide_instance_runs_to_steady_state_with_retirement():
    """run_to_steady over a batch holding a one-block instance and a large-set instance:
    both reach r < 1e-9 and the converged one is retired (not advanced) while the other
    keeps stepping; the large-set steady state satisfies the oracle's L[F] = 0 to the
    residual level."""
    from paper_1708_05944_amd import Batch
    o, d = _pair(N_R=6, ax1=(1, 20, 4), ax2=(0, 25, 4), Kn=0.5, u_in=0.2)   # 1000 velocities, 65 nodes
    o2, d2 = _pair(N_R=16, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.1, u_in=0.1)
    b = Batch([d, d2])
    steps, r, ok = b.run_to_steady(1e-9, 200000, 500)
    _say(f"steps {steps}, residuals {r}")
    assert ok and (r < 1e-9).all() and (steps > 0).all()
    F = b.instance_view(b.get_state(), 0).copy()
    L, _ = o.L(F)
    assert np.abs(L).max() <= 1e-6 * np.abs(F).max()
    b.close()


# ---------------------------------------------------------------- f-tilde formulation
FTILDE_CASES = [
    # the paper's Fig. komissarov set-up: cylinders at rest, H(4;5)^2, stretched cells
    dict(N_R=16, ax1=(0, 5, 4), ax2=(0, 5, 4), Kn=1e-3, tau_model=2, u_in=0.0, A=0.95, delta=0.5, form=1),
    # moving inner wall, half-range radial axis, equal cells, hotter outer wall
    dict(N_R=12, ax1=(1, 4, 3), ax2=(0, 6, 4), Kn=0.2, u_in=0.3, T_out=1.1, form=1),
]


@pytest.mark.parametrize("case", FTILDE_CASES)
def test_ftilde_operator_and_steps_match_oracle(case):
    """The f-tilde formulation (Sec. III, Eq. boltz_cons; the paper's comparison scheme)
    on the four-launch stage: L and 10 RK3 steps against the oracle's f-tilde operator."""
    from paper_1708_05944_amd import Batch
    _say(f"case {case}")
    o, d = _pair(**dict(case))
    b = Batch([d])
    F = _perturbed(o, 5)
    b.set_state(F.ravel())
    err = _relerr(b.instance_view(b.apply_L(), 0), o.L(F)[0])
    _say(f"f-tilde L rel err {err:.2e}")
    assert err <= TOL
    b.step(10)
    err = _relerr(b.instance_view(b.get_state(), 0), o.step(F, b.info[0]["dt"], 10))
    _say(f"f-tilde 10 steps rel err {err:.2e}")
    assert err <= TOL
    b.close()


def test_rest_state_ftilde_vs_chi_on_the_gpu():
    """Sec. V.C.2 (Fig. komissarov): cylinders at rest on stretched cells; from the rest
    Maxwellian the chi form stays at n = 1 to rounding over 400 steps, the f-tilde form
    redistributes particles (the same deviation as the oracle's, to 1e-10)."""
    from paper_1708_05944_amd import Batch
    dev = {}
    for form in (0, 1):
        case = dict(FTILDE_CASES[0], form=form)
        o, d = _pair(**case)
        d.dt = 1e-3
        b = Batch([d])
        b.init_equilibrium(0, 1.0, 0.0, 0.0, 1.0)
        b.step(400)
        n = b.moments(0)["n"]
        dev[form] = np.abs(n - 1.0).max()
        if form == 1:
            want = o.moments(o.step(o.equilibrium(1.0, 0.0, 0.0, 1.0), 1e-3, 400))["n"]
            assert np.abs(n - want).max() <= 1e-10
        b.close()
    _say(f"max |n - 1| after 400 steps: chi {dev[0]:.1e}, f-tilde {dev[1]:.1e}")
    assert dev[0] <= 1e-12 and dev[1] >= 1e-3
