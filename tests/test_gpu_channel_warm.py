"""Learned warm start of expanding channels (a reduced channel family: 32 x 8 cells,
HH(3;4) x H(4;8), Kn 0.04-0.25, r 1.5-3): the surrogate (the library's MLP kernels)
trained on steady states the channel solver produced, its warm state against the
oracle's local equilibrium of the same predicted fields, and what it gains over the
cold start."""
import sys

import numpy as np
import pytest

from oracle.channel import ChannelOracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle(d):
    kw = {k: getattr(d, k) for k in ("xi_in", "xi_out", "r", "L", "ax1", "ax2", "Kn", "tau_model", "n_in", "n_out",
                                      "T_w", "weno_eps")}
    return ChannelOracle(NL=d.N_lambda, NX=d.N_xi, **kw)


def test_channel_warm_start_state_and_gain():
    """Train on 16 channels (seed 11), start 8 held-out ones (seed 12) from rest and from
    the surrogate, FP64 to r < 1e-10: the warm state of every held-out instance is the
    oracle's local equilibrium of the network's fields (1e-13), the warm runs lose no
    instance the cold runs converge, and need fewer steps in total (a non-converged
    instance counting the whole budget)."""
    import torch

    from paper_1708_05944_amd import Channel, surrogate, workloads
    tr = workloads.channel_surrogate_descs(16, workloads.CHANNEL_SURROGATE_TRAIN_SEED)
    ho = workloads.channel_surrogate_descs(8, workloads.CHANNEL_SURROGATE_HELDOUT_SEED)
    X, Y, st = surrogate.channel_steady_samples(tr, max_steps=150_000, log=_say)
    _say(f"training solves {st}")
    assert st["converged"] >= 12
    mlp, losses = surrogate.train(X, Y, epochs=300, batch=256, lr=1e-3)
    _say(f"final loss {losses[-1]:.3e}")
    assert losses[-1] < 0.1 * losses[0]
    c = Channel(ho)
    surrogate.channel_warm_start(c, mlp)
    for b in range(c.B):
        Yb = mlp.forward(surrogate.channel_features(ho[b], c.info[b]), bf16=True)
        want = _oracle(ho[b]).equilibrium(*surrogate.channel_fields(Yb, c.info[b]))
        got = c.get_instance_state(b)
        err = max(np.abs(got[d] - want[d]).max() / np.abs(want[d]).max() for d in range(2))
        assert err <= 1e-13, (b, err)
    c.close()
    runs = {}
    for name, warm in (("cold", False), ("warm", True)):
        c = Channel(ho)
        if warm:
            surrogate.channel_warm_start(c, mlp)
        conv, r, fell = surrogate.channel_run(c, 1e-10, 150_000, stall_window=40_000 if warm else None,
                                              warm=np.full(c.B, warm))
        torch.cuda.synchronize()
        runs[name] = np.where(conv >= 0, conv, 150_000), int((conv >= 0).sum())
        _say(f"{name}: converged {runs[name][1]}/8, steps {list(conv)}, cold restarts {list(fell)}")
        c.close()
    mlp.close()
    assert runs["warm"][1] >= runs["cold"][1]
    assert runs["warm"][0].sum() < runs["cold"][0].sum()
