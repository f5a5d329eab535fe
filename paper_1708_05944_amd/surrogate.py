"""Learned warm start: training data from the library's own steady states, training on
the GPU through the library's kernels, and warm-started runs.  Marshalling only: every
numerical step (solves, moments, forward / backward passes, Adam, inference, initial
states) runs in libvlb.so."""
from __future__ import annotations

import time

import numpy as np

from . import workloads
from .vlb import VLB_FP64, Batch, Mlp


def run_to_steady(batch, tol: float, max_steps: int, check_every: int = 500, chunk: int = 50_000, log=None,
                  times=None):
    """batch.run_to_steady in chunks of `chunk` steps (a progress line per chunk through
    `log`); returns (steps at convergence per instance, -1 if not converged; last
    residuals; all converged).  With `times` (an array of B), the wall-clock seconds
    from the call to the end of the chunk in which each instance converged."""
    import torch
    conv = np.full(batch.B, -1, dtype=np.int64)
    done, r = 0, None
    t0 = time.perf_counter()
    while done < max_steps:
        n = min(chunk, max_steps - done)
        steps, r, ok = batch.run_to_steady(tol, n, check_every)
        torch.cuda.synchronize()
        new = (conv < 0) & (steps >= 0)
        conv[new] = done + steps[new]
        if times is not None:
            times[new] = time.perf_counter() - t0
        done += n
        if log:
            log(f"  {done} steps: {int((conv >= 0).sum())}/{batch.B} below {tol:g}, largest residual {r.max():.2e}")
        if (conv >= 0).all():
            break
    return conv, r, bool((conv >= 0).all())


def warm_start_comparison(train_descs, heldout_descs, epochs: int = 1000, batch: int = 256, lr: float = 1e-3,
                          probe: int = 500, max_steps: int = 200_000, chunk: int = 5_000, log=None,
                          keep_fields: bool = False):
    """The learned warm start end to end: steady states of the training instances ->
    samples -> trained network -> held-out instances run to r < 1e-10 from the cold rest
    state in FP64 (the plain solver) and from the warm start in mixed precision.
    Returns a dict of timings and per-instance step counts; times of a run are taken at
    the chunk in which its last converging instance converged."""
    from .vlb import VLB_MIXED
    X, T, st = steady_samples(train_descs, tol=1e-10, max_steps=max_steps, log=log)
    t0 = time.perf_counter()
    mlp, losses = train(X, T, epochs=epochs, batch=batch, lr=lr)
    t_train = time.perf_counter() - t0
    out = dict(training_solves=st, samples=int(len(X)), train_seconds=t_train, epochs=epochs,
               final_loss=float(losses[-1]))
    runs = {}
    for name, prec, warm in (("cold_fp64", VLB_FP64, False), ("warm_mixed", VLB_MIXED, True)):
        b = Batch(heldout_descs, precision=prec)
        b.autotune(3)
        b.init_equilibrium(-1, 1.0, 0.0, 0.0, 1.0)
        times = np.full(b.B, np.nan)
        t0 = time.perf_counter()
        used = b.warm_start(mlp, probe) if warm else np.zeros(b.B, np.int32)
        t_ws = time.perf_counter() - t0
        steps, r, ok = run_to_steady(b, 1e-10, max_steps, chunk=chunk, log=log, times=times)
        runs[name] = dict(steps=steps, times=times + t_ws, used=used, warm_start_seconds=t_ws,
                          fp32_steps=b.fp32_steps() if warm else 0)
        if keep_fields:
            runs[name]["fields"] = [b.moments(i) for i in range(b.B)]
        b.close()
    both = (runs["cold_fp64"]["steps"] >= 0) & (runs["warm_mixed"]["steps"] >= 0)
    c, w = runs["cold_fp64"], runs["warm_mixed"]
    out.update(heldout=len(heldout_descs), converged_cold=int((c["steps"] >= 0).sum()),
               converged_warm=int((w["steps"] >= 0).sum()), converged_both=int(both.sum()),
               warm_used=int(w["used"].sum()), probe_steps=probe,
               steps_cold=int(c["steps"][both].sum()), steps_warm=int(w["steps"][both].sum() + 2 * probe * both.sum()),
               seconds_cold=float(np.nanmax(c["times"][both])) if both.any() else None,
               seconds_warm=float(np.nanmax(w["times"][both])) if both.any() else None,
               warm_start_seconds=w["warm_start_seconds"], fp32_steps=int(w["fp32_steps"]),
               per_instance_steps_cold=[int(x) for x in c["steps"]],
               per_instance_steps_warm=[int(x) for x in w["steps"]])
    if out["seconds_cold"] and out["seconds_warm"]:
        out["speedup"] = out["seconds_cold"] / out["seconds_warm"]
    if keep_fields:
        out["fields"] = {k: v["fields"] for k, v in runs.items()}
        out["converged_mask"] = both
    mlp.close()
    return out


def steady_samples(descs, tol: float = 1e-10, max_steps: int = 2_000_000, check_every: int = 500, log=None):
    """Run a batch of instances to steady state (FP64; converged instances retire) and
    return the surrogate samples (X, T) of the cells of the instances that converged,
    with the solve's statistics."""
    b = Batch(descs, precision=VLB_FP64)
    b.autotune(3)
    b.init_equilibrium(-1, 1.0, 0.0, 0.0, 1.0)
    t0 = time.perf_counter()
    steps, r, ok = run_to_steady(b, tol, max_steps, check_every, log=log)
    secs = time.perf_counter() - t0
    X, T = b.surrogate_samples()
    keep = np.repeat(steps >= 0, [i["N_R"] for i in b.info])
    b.close()
    return X[keep], T[keep], dict(seconds=secs, max_steps=int(steps.max()), converged=int((steps >= 0).sum()),
                                  instances=len(descs))


def train(X, T, epochs: int = 400, batch: int = 512, lr: float = 1e-3, width: int = 128, depth: int = 3,
          seed: int = 0, init_seed: int = 0):
    """Train a surrogate on (X, T) with Adam, one fresh permutation per epoch; returns the
    network and its per-epoch mean losses."""
    mlp = Mlp(workloads.mlp_init_params(width, depth, init_seed), width, depth)
    losses = [mlp.train(X, T, order, batch, lr) for order in workloads.epoch_orders(len(X), epochs, seed)]
    return mlp, np.array(losses)
