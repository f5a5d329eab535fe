"""Parity at the benchmarked sizes, in the launch configuration `bench.py` times.

* Batched Couette sweep (256 instances, 20.9 M site-velocities): the batch is built and
  autotuned as the bench does, advanced from rest, then one more step is compared, on a
  sample of instances that covers the extremes of grid and velocity-set size, with the
  oracle's RK3 step from the same state -- FP64 at 1e-12, mixed precision (FP32 stage
  kernels on weight-scaled populations) at 2e-6 (FP32 rounding, as for the operator).
* Expanding channel 512 x 128 cells, HH(4;8) x H(4;16): every cell, both the operator
  L[F] and one RK3 step, against the oracle at 1e-12 (FP64), and one FP32 step against
  the oracle's step from the FP32-rounded state at 2e-6 (mixed).  The grid is wider than
  one 32-cell lambda strip, so this covers the multi-strip traversal of the stage kernel.
"""
import sys

import numpy as np
import pytest

from oracle.couette import CouetteOracle

pytestmark = pytest.mark.gpu

_ORACLE_KEYS = ("R_in", "R_out", "N_R", "ax1", "ax2", "Kn", "tau_model", "u_in", "T_in", "u_out", "T_out", "A",
                "delta", "weno_eps")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relerr(a, b):
    a = np.asarray(a).reshape(2, -1)
    b = np.asarray(b).reshape(2, -1)
    return max(np.abs(a[d] - b[d]).max() / np.abs(b[d]).max() for d in range(2))


def _sample(descs):
    """Instances with the most / fewest velocities and cells, plus every eighth."""
    nv = [d.ax1[1] * (2 if d.ax1[0] == 1 else 1) * d.ax2[1] * (2 if d.ax2[0] == 1 else 1) for d in descs]
    nr = [d.N_R for d in descs]
    picks = {int(np.argmax(nv)), int(np.argmin(nv)), int(np.argmax(nr)), int(np.argmin(nr)),
             int(np.argmax(np.array(nv) * np.array(nr)))}
    picks.update(range(0, len(descs), 8))
    return sorted(picks)


def _sweep_step_parity(precision, tol):
    import torch
    from paper_1708_05944_amd import Batch, workloads
    descs = workloads.couette_sweep()
    b = Batch(descs, precision=precision)
    b.step(1)
    tile, _ = b.autotune(3)
    b.step(4)
    torch.cuda.synchronize()
    F = b.get_state()
    b.step(1)
    G = b.get_state()
    _say(f"sweep precision {precision}: tile {tile}, state of {F.size} values")
    worst = 0.0
    for i in _sample(descs):
        d = descs[i]
        o = CouetteOracle(**{k: getattr(d, k) for k in _ORACLE_KEYS})
        want = o.step(b.instance_view(F, i).copy(), b.info[i]["dt"], 1)
        err = _relerr(b.instance_view(G, i), want)
        worst = max(worst, err)
        assert err <= tol, (i, d, err)
    _say(f"sweep precision {precision}: {len(_sample(descs))} sampled instances, worst rel err {worst:.2e}")
    b.close()


def test_sweep_fp64_full_size_matches_oracle():
    _sweep_step_parity(0, 1e-12)


def test_sweep_mixed_full_size_matches_oracle():
    from paper_1708_05944_amd import VLB_MIXED
    _sweep_step_parity(VLB_MIXED, 2e-6)


def test_channel_full_size_matches_oracle():
    import torch
    from oracle.channel import ChannelOracle
    from paper_1708_05944_amd import Channel, ChannelDesc
    kw = dict(xi_in=-4.0, xi_out=12.0, r=2.0, L=4.0, ax1=(1, 8, 4), ax2=(0, 16, 4), Kn=0.05, tau_model=1, n_in=1.1,
              n_out=0.9, T_w=1.0)
    c = Channel([ChannelDesc(N_lambda=128, N_xi=512, **kw)])
    o = ChannelOracle(NL=128, NX=512, **kw)
    c.step(3)
    torch.cuda.synchronize()
    F = c.instance_view(c.get_state(), 0).copy()
    L = c.instance_view(c.apply_L(), 0)
    Lw, _, _ = o.L(F)
    err = _relerr(L, Lw)
    _say(f"channel 512 x 128 operator rel err {err:.2e}")
    assert err <= 1e-12
    c.step(1)
    G = c.instance_view(c.get_state(), 0)
    want = o.step(F, c.info[0]["dt"], 1)
    err = _relerr(G, want)
    _say(f"channel 512 x 128 step rel err {err:.2e}")
    assert err <= 1e-12
    c.close()


def test_channel_mixed_full_size_matches_oracle():
    import torch
    from oracle.channel import ChannelOracle
    from paper_1708_05944_amd import VLB_MIXED, Channel, ChannelDesc
    kw = dict(xi_in=-4.0, xi_out=12.0, r=2.0, L=4.0, ax1=(1, 8, 4), ax2=(0, 16, 4), Kn=0.05, tau_model=1, n_in=1.1,
              n_out=0.9, T_w=1.0)
    c = Channel([ChannelDesc(N_lambda=128, N_xi=512, **kw)], precision=VLB_MIXED)
    o = ChannelOracle(NL=128, NX=512, **kw)
    c.step(3)
    torch.cuda.synchronize()
    F = c.instance_view(c.get_state(), 0).copy()   # FP32 state in FP64 (moves it to FP64)
    c.step(1)                                       # back to FP32 (exactly), one FP32 step
    G = c.instance_view(c.get_state(), 0)
    want = o.step(F, c.info[0]["dt"], 1)
    err = _relerr(G, want)
    _say(f"channel 512 x 128 FP32 step rel err {err:.2e}")
    assert err <= 2e-6
    c.close()


def _channel_sweep_parity(precision, tol):
    """The 64-channel sweep (seed 3: 64..256 x 256..1024 cells, 256..512 velocities, both
    velocity-tile classes) advanced together; the smallest instance of each tile class is
    compared with the oracle's step from the same state."""
    import torch
    from oracle.channel import ChannelOracle
    from paper_1708_05944_amd import Channel, workloads
    descs = workloads.channel_sweep()
    c = Channel(descs, precision=precision)
    c.step(2)
    torch.cuda.synchronize()
    size = [d.N_lambda * d.N_xi * d.ax1[1] for d in descs]
    picks = []
    for cls in (lambda d: d.ax1[1] <= 8, lambda d: d.ax1[1] > 8):
        idx = [i for i, d in enumerate(descs) if cls(d)]
        if idx:
            picks.append(min(idx, key=lambda i: size[i]))
    _say(f"channel sweep precision {precision}: {c.state_size} values, checking instances {picks}")
    states = {i: c.get_instance_state(i) for i in picks}   # FP64 (for a mixed batch: its FP32 state)
    c.step(1)
    # every instance (the batch holds more than 2^32 populations) has a finite residual
    assert np.isfinite(c.residual()).all()
    for i in picks:
        d = descs[i]
        G = c.get_instance_state(i)
        o = ChannelOracle(NL=d.N_lambda, NX=d.N_xi, ax1=d.ax1, ax2=d.ax2, Kn=d.Kn, tau_model=d.tau_model, r=d.r, L=d.L,
                          xi_in=d.xi_in, xi_out=d.xi_out, n_in=d.n_in, n_out=d.n_out, T_w=d.T_w)
        want = o.step(states[i], c.info[i]["dt"], 1)
        err = _relerr(G, want)
        _say(f"instance {i} ({d.N_lambda} x {d.N_xi}, ax1 {d.ax1}): rel err {err:.2e}")
        assert err <= tol
    c.close()


def test_channel_sweep_full_size_mixed_matches_oracle():
    from paper_1708_05944_amd import VLB_MIXED
    _channel_sweep_parity(VLB_MIXED, 2e-6)


def test_channel_sweep_full_size_fp64_matches_oracle():
    _channel_sweep_parity(0, 1e-12)
