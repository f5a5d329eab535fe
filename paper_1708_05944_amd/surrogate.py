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


def heldout_runs(heldout_descs, mlp, probe: int = 500, max_steps: int = 200_000, chunk: int = 5_000,
                 check_every: int = 500, stall_window: int = 10_000, log=None, keep_fields: bool = False,
                 legs=(("cold_fp64", 0, False), ("warm_fp64", 0, True), ("cold_mixed", 1, False),
                       ("warm_mixed", 1, True))):
    """The held-out instances run to r < 1e-10 from the cold rest state and from the
    surrogate's warm start, each in FP64 and in mixed precision (defect correction).
    Per leg: steps at convergence per instance (-1 if not converged), wall-clock seconds
    of the whole batch (until every instance converged, or max_steps), the warm starts
    kept by the acceptance probe, the instances restarted cold by the stall watch, and for
    the mixed legs the FP32 correction steps summed over the instances and the instances
    that left the correction for FP64 steps for good."""
    import torch
    from .vlb import VLB_MIXED
    runs = {}
    for name, prec, warm in legs:
        b = Batch(heldout_descs, precision=VLB_MIXED if prec else VLB_FP64)
        b.autotune(3)
        b.init_equilibrium(-1, 1.0, 0.0, 0.0, 1.0)
        b.set_stall_window(stall_window)
        torch.cuda.synchronize()
        times = np.full(b.B, np.nan)
        t0 = time.perf_counter()
        used = b.warm_start(mlp, probe) if warm else np.zeros(b.B, np.int32)
        t_ws = time.perf_counter() - t0
        if log:
            log(f" {name}: {len(heldout_descs)} instances, warm starts kept {int(used.sum())}")
        steps, r, ok = run_to_steady(b, 1e-10, max_steps, check_every=check_every, chunk=chunk, log=log, times=times)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        on_warm, fell = b.warm_report()
        _, fp64_from, n32 = b.mixed_report()
        runs[name] = dict(steps=steps, times=times + t_ws, seconds=secs, used=used, warm_start_seconds=t_ws,
                          fp32_steps=int(n32.sum()), fp64_kept=int((fp64_from >= 0).sum()), fallback_at=fell,
                          converged=int((steps >= 0).sum()), probe_steps=2 * probe * int(warm))
        if keep_fields:
            runs[name]["fields"] = [b.moments(i) for i in range(b.B)]
        b.close()
    return runs


def summarise(runs, max_steps: int):
    """Honest totals of heldout_runs: an instance that did not converge counts max_steps
    steps (and the batch's whole wall time); speed-ups compare the legs over all
    instances; fp32_share = FP32 correction steps / all steps of the instances."""
    out = {}
    for name, rr in runs.items():
        st = np.where(rr["steps"] >= 0, rr["steps"], max_steps)
        out[name] = dict(converged=rr["converged"], instances=len(st), steps_total=int(st.sum() + rr["probe_steps"]),
                         seconds=float(rr["seconds"]), warm_used=int(np.sum(rr["used"])),
                         cold_restarts=int((rr["fallback_at"] >= 0).sum()), fp32_steps=int(rr["fp32_steps"]),
                         fp32_share=float(rr["fp32_steps"] / st.sum()), fp64_kept=int(rr["fp64_kept"]),
                         per_instance_steps=[int(x) for x in rr["steps"]])
    pairs = (("warm_fp64", "cold_fp64"), ("warm_mixed", "cold_mixed"), ("warm_mixed", "cold_fp64"),
             ("cold_mixed", "cold_fp64"))
    for w, c in pairs:
        if w in out and c in out:
            out[f"speedup_{w}_vs_{c}"] = out[c]["seconds"] / out[w]["seconds"]
            out[f"step_ratio_{w}_vs_{c}"] = out[c]["steps_total"] / out[w]["steps_total"]
    return out


def warm_start_comparison(train_descs, heldout_descs, epochs: int = 1000, batch: int = 256, lr: float = 1e-3,
                          probe: int = 500, max_steps: int = 200_000, chunk: int = 5_000, log=None,
                          keep_fields: bool = False, stall_window: int = 10_000, extra=None):
    """The learned warm start end to end: steady states of the training instances ->
    samples -> trained network -> held-out instances run to r < 1e-10 cold and warm, in
    FP64 and mixed precision (heldout_runs, summarise).  extra: {label: descriptors} of
    further held-out sets run the same way with the same network (out["extra"][label])."""
    X, T, st = steady_samples(train_descs, tol=1e-10, max_steps=max_steps, log=log)
    t0 = time.perf_counter()
    mlp, losses = train(X, T, epochs=epochs, batch=batch, lr=lr)
    t_train = time.perf_counter() - t0
    out = dict(training_solves=st, samples=int(len(X)), train_seconds=t_train, epochs=epochs,
               final_loss=float(losses[-1]), heldout=len(heldout_descs), probe_steps=probe, max_steps=max_steps,
               stall_window=stall_window)
    runs = heldout_runs(heldout_descs, mlp, probe=probe, max_steps=max_steps, chunk=chunk, log=log,
                        keep_fields=keep_fields, stall_window=stall_window)
    out.update(summarise(runs, max_steps))
    if keep_fields:
        out["fields"] = {k: v["fields"] for k, v in runs.items()}
        out["steps"] = {k: v["steps"] for k, v in runs.items()}
    for label, descs in (extra or {}).items():
        if log:
            log(f" held-out set {label}")
        rx = heldout_runs(descs, mlp, probe=probe, max_steps=max_steps, chunk=chunk, log=log,
                          stall_window=stall_window)
        out.setdefault("extra", {})[label] = summarise(rx, max_steps)
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
