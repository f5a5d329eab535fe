"""The no-allocation entry point (vlb_couette_step_noalloc) against the batch entry point
it mirrors (vlb_set_state + vlb_step + vlb_residual on a batch created from the same
descriptors): the same kernels on the same state, so the states must agree to the FP64
parity bar (1e-12 of the largest population; they are expected to be bitwise equal) and
the residuals to 1e-12 relative.  Two calls in a row share the library's scratch array;
the second has a smaller input (fewer instances, cells and velocities), so stale
contents of the first call would show."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _perturbed_state(batch, seed):
    rng = np.random.default_rng(seed)
    for b, i in enumerate(batch.info):
        x = (np.arange(i["N_R"]) + 0.5) / i["N_R"]
        batch.init_equilibrium(b, 1.0 + 0.1 * np.sin(2 * np.pi * x), 0.05 * np.cos(np.pi * x),
                               0.1 * (1 - x), 1.0 + 0.05 * x * x)
    F = batch.get_state()
    return F * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, F.shape))


def _compare(descs, nsteps, seed):
    import torch
    from paper_1708_05944_amd import Batch, couette_step_noalloc
    ref = Batch(descs)
    F0 = _perturbed_state(ref, seed)
    ref.set_state(F0)
    ref.step(nsteps)
    want = ref.get_state()
    r_want = ref.residual()
    ref.close()
    Ft = torch.from_numpy(F0.copy()).to("cuda")
    r_got = couette_step_noalloc(descs, Ft, nsteps)
    torch.cuda.synchronize()
    got = Ft.cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    rerr = np.abs(r_got - r_want).max() / np.abs(r_want).max()
    _say(f"  {len(descs)} instance(s), {nsteps} steps: state err {err:.2e}, residual err {rerr:.2e}")
    assert err <= 1e-12 and rerr <= 1e-12, (err, rerr)


def test_noalloc_matches_batch_step_on_two_calls():
    from paper_1708_05944_amd import CouetteDesc
    first = [CouetteDesc(N_R=40, ax1=(1, 3, 2), ax2=(0, 5, 3), Kn=0.3, u_in=0.2),
             CouetteDesc(N_R=25, ax1=(1, 4, 2), ax2=(0, 4, 2), Kn=0.05, u_in=0.1, A=0.9, delta=0.4, u_out=-0.05),
             CouetteDesc(N_R=70, R_out=1.6, ax1=(1, 6, 4), ax2=(0, 9, 4), Kn=1.0, u_in=0.4, T_out=1.1)]
    second = [CouetteDesc(N_R=12, ax1=(1, 2, 1), ax2=(0, 3, 2), Kn=0.5, u_in=0.3)]
    _say("no-alloc call 1: three instances, 23 steps")
    _compare(first, 23, 1)
    _say("no-alloc call 2: one smaller instance, 7 steps")
    _compare(second, 7, 2)
