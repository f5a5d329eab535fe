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


# ---------------------------------------------------------------- expanding channels
# The same network (4 -> 128 -> 128 -> 128 -> 4, the library's MLP kernels) maps a channel
# cell's (log10 Kn, r, xi, lambda), each mapped affinely to [-1, 1], to its steady
# (n - 1, u^lambda, u^xi, T - 1) times CH_SCALE (outputs of order one).
CH_SCALE = np.array([10.0, 5.0, 5.0, 50.0])


def channel_features(desc, info) -> np.ndarray:
    """Surrogate inputs of every cell of one channel ([N_xi * N_lambda][4] float32, xi-major
    like the state): cell centres of the equal xi and lambda cells (full width, A = 0)."""
    if desc.half or desc.A != 0:
        raise ValueError("the channel surrogate covers full-width channels on equal cells")
    NX, NL = info["N_xi"], info["N_lambda"]
    xi = desc.xi_in + (np.arange(NX) + 0.5) * (desc.xi_out - desc.xi_in) / NX
    lam = -1.0 + (np.arange(NL) + 0.5) * 2.0 / NL
    X, L = np.meshgrid(xi, lam, indexing="ij")
    lo, hi = np.log10(workloads.CHANNEL_SURROGATE_KN[0]), np.log10(workloads.CHANNEL_SURROGATE_KN[1])
    rlo, rhi = workloads.CHANNEL_SURROGATE_R
    cols = [np.full(X.shape, (np.log10(desc.Kn) - 0.5 * (lo + hi)) / (0.5 * (hi - lo))),
            np.full(X.shape, (desc.r - 0.5 * (rlo + rhi)) / (0.5 * (rhi - rlo))),
            (X - 0.5 * (desc.xi_in + desc.xi_out)) / (0.5 * (desc.xi_out - desc.xi_in)), L]
    return np.stack([c.ravel() for c in cols], axis=-1).astype(np.float32)


def channel_targets(m) -> np.ndarray:
    return (np.stack([m["n"].ravel() - 1.0, m["u1"].ravel(), m["u2"].ravel(), m["T"].ravel() - 1.0], axis=-1)
            * CH_SCALE).astype(np.float32)


def channel_fields(Y, info):
    """(n, u^lambda, u^xi, T) per cell ([N_xi][N_lambda] each) from surrogate outputs."""
    Y = np.asarray(Y, dtype=np.float64) / CH_SCALE
    shp = (info["N_xi"], info["N_lambda"])
    return (1.0 + Y[:, 0]).reshape(shp), Y[:, 1].reshape(shp), Y[:, 2].reshape(shp), (1.0 + Y[:, 3]).reshape(shp)


def channel_run(c, tol, max_steps, chunk=10_000, check_every=1000, stall_window=None, warm=None, log=None,
                patience=None):
    """Run a channel batch (FP64) to r < tol in chunks; returns (steps at convergence per
    instance or -1, last residuals, cold restarts per instance (step or -1)).  With
    stall_window, an instance started warm whose residual sets no new low (by 1 %) for
    stall_window steps is restarted from the rest state (the plain solver's residual
    decides, the cold start is the fallback).  With patience, the run also stops once no
    instance has converged for that many steps (for training solves, where the instances
    that do converge are what is wanted)."""
    B = c.B
    conv = np.full(B, -1, dtype=np.int64)
    fell = np.full(B, -1, dtype=np.int64)
    best = np.full(B, np.inf)
    best_at = np.zeros(B, dtype=np.int64)
    warm = np.zeros(B, bool) if warm is None else np.asarray(warm, bool).copy()
    done, r, last_new = 0, None, 0
    while done < max_steps and (conv < 0).any():
        n = min(chunk, max_steps - done)
        steps, r, ok = c.run_to_steady(tol, n, check_every)
        new = (conv < 0) & (steps >= 0)
        conv[new] = done + steps[new]
        done += n
        if new.any():
            last_new = done
        if patience and (conv >= 0).any() and done - last_new >= patience:
            break
        for b in np.flatnonzero((conv < 0) & warm):
            if r[b] < 0.99 * best[b]:
                best[b], best_at[b] = r[b], done
            elif stall_window and done - best_at[b] >= stall_window:
                d = c.descs[b]
                c.init_equilibrium(b, 1.0, 0.0, 0.0, d.T_w)
                warm[b] = False
                fell[b] = done
        if log:
            log(f"  {done} steps: {int((conv >= 0).sum())}/{B} below {tol:g}, largest residual {r.max():.2e}")
    return conv, r, fell


def channel_steady_samples(descs, tol=1e-10, max_steps=400_000, log=None):
    """Steady states of a channel batch (FP64, from rest) and the surrogate samples of the
    cells of the instances that converged."""
    from .vlb import Channel
    c = Channel(descs)
    t0 = time.perf_counter()
    conv, r, _ = channel_run(c, tol, max_steps, log=log, patience=30_000)
    secs = time.perf_counter() - t0
    X, Y = [], []
    for b in np.flatnonzero(conv >= 0):
        X.append(channel_features(descs[b], c.info[b]))
        Y.append(channel_targets(c.moments(b)))
    c.close()
    return (np.concatenate(X), np.concatenate(Y),
            dict(seconds=secs, converged=int((conv >= 0).sum()), instances=len(descs), max_steps=int(conv.max())))


def channel_warm_start(c, mlp, bf16: bool = True):
    """Set every instance of a channel batch to the local equilibrium of the surrogate's
    fields (network inference on the device, the state built on the device)."""
    for b in range(c.B):
        Y = mlp.forward(channel_features(c.descs[b], c.info[b]), bf16=bf16)
        c.init_equilibrium(b, *channel_fields(Y, c.info[b]))


def channel_warm_comparison(train_descs, heldout_descs, epochs: int = 300, batch: int = 256, lr: float = 1e-3,
                            max_steps: int = 200_000, stall_window: int = 40_000, log=None):
    """The learned channel warm start end to end: steady states of the training channels ->
    samples -> trained network -> held-out channels run to r < 1e-10 from rest and from the
    surrogate (FP64), with honest totals (an instance that did not converge counts
    max_steps steps and the leg's whole wall time)."""
    import torch
    from .vlb import Channel
    X, Y, st = channel_steady_samples(train_descs, max_steps=max_steps, log=log)
    t0 = time.perf_counter()
    mlp, losses = train(X, Y, epochs=epochs, batch=batch, lr=lr)
    t_train = time.perf_counter() - t0
    out = dict(training_solves=st, samples=int(len(X)), train_seconds=t_train, epochs=epochs,
               final_loss=float(losses[-1]), heldout=len(heldout_descs), max_steps=max_steps,
               stall_window=stall_window)
    for name, warm in (("cold_fp64", False), ("warm_fp64", True)):
        c = Channel(heldout_descs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if warm:
            channel_warm_start(c, mlp)
        conv, r, fell = channel_run(c, 1e-10, max_steps, stall_window=stall_window if warm else None,
                                    warm=np.full(c.B, warm), log=log)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        st_ = np.where(conv >= 0, conv, max_steps)
        out[name] = dict(converged=int((conv >= 0).sum()), instances=c.B, steps_total=int(st_.sum()),
                         seconds=secs, cold_restarts=int((fell >= 0).sum()),
                         per_instance_steps=[int(x) for x in conv])
        c.close()
    out["speedup_warm_fp64_vs_cold_fp64"] = out["cold_fp64"]["seconds"] / out["warm_fp64"]["seconds"]
    out["step_ratio_warm_fp64_vs_cold_fp64"] = out["cold_fp64"]["steps_total"] / out["warm_fp64"]["steps_total"]
    mlp.close()
    return out
