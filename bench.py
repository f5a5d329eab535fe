"""Throughput benchmark of the vielbein-LB hot path on one MI355X.

Workload (seeded, synthetic): the batched circular-Couette sweep -- 256 instances with
Kn = 10^U(-2,1), wall speed U(0.05, 0.5), radius ratio U(0.3, 0.8), 64..512 cells, and
HH(N;Q_R) x H(N;Q_phi) velocity sets whose orders grow with Kn (32..640 velocities),
all advanced together by the library's RK3 stage kernels, in mixed precision (FP32
stage kernels on weight-scaled populations; the headline) and in FP64.  One "step" is
one full third-order Runge-Kutta step of every instance.

Prints one JSON line: site-velocity updates per second (sum over instances of
cells x velocities x steps / wall time), the roofline of the dominant stage-kernel
instantiation (HIP events around each of its launches over the timed region; bytes =
algorithmic HBM traffic, one read of the stage input, one read of F_n in stages 2 and
3, one write, per population) and the CPU oracle's rate on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak with plain (non-packed) FMAs, 256 CUs x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz;
# the library is built with packed FP32 instructions disabled, so 157.3 TFLOP/s is out of reach
VALU_FP32_TFLOPS = 78.6
VALU_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "couette_stage_traffic.json")


def stage_flops(descs) -> float:
    """Algorithmic flops of one RK stage over the batch: per site-velocity, two
    distributions x (WENO-5 face ~54, force 2 x 2 Q_R + 2 Q_phi + 5, BGK/combine ~8),
    plus ~13 for moments and the equilibrium factor product."""
    tot = 0.0
    for d in descs:
        n1 = d.ax1[1] * (2 if d.ax1[0] == 1 else 1)
        n2 = d.ax2[1] * (2 if d.ax2[0] == 1 else 1)
        tot += d.N_R * n1 * n2 * (2 * (54 + 2 * n1 + 2 * n2 + 5 + 8) + 13)
    return tot


def channel_stage_flops(cells: int, q1: int, q2: int) -> float:
    """Algorithmic flops of one channel RK stage: per site-velocity, two distributions x
    (four WENO-5 faces ~4 x 54, the four momentum-derivative contractions 2 (2 Q1 + 2 Q2),
    advection, BGK and combination ~18), plus ~13 for moments and the equilibrium."""
    return cells * q1 * q2 * (2 * (4 * 54 + 4 * (q1 + q2) + 18) + 13)


def roofline(kernel: str, ms: float, alg_bytes: float, alg_flops: float, peak_tflops: float, traffic, **extra):
    """Roofline record of one launch of `kernel`: algorithmic bytes and flops per launch over
    its mean duration.  The bound is the ceiling the kernel's arithmetic intensity reaches
    first: ALU above the ridge (peak flop rate / HBM bandwidth), HBM below it; the other
    ceiling is reported beside it."""
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    tfs = alg_flops / (ms * 1e-3) / 1e12
    ridge = peak_tflops * 1e3 / HBM_PEAK_GBS
    intensity = alg_flops / alg_bytes
    hbm = {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "alg_bytes_per_launch": alg_bytes}
    alu = {"achieved": tfs, "peak": peak_tflops, "unit": "TFLOP/s", "frac": tfs / peak_tflops,
           "alg_flops_per_launch": alg_flops}
    main, bound = (alu, "alu") if intensity > ridge else (hbm, "hbm")
    rec = {"bound": bound, "achieved": main["achieved"], "peak": main["peak"], "unit": main["unit"],
           "frac": main["frac"], "traffic": traffic, "kernel": kernel, "avg_launch_ms": ms,
           "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge, "hbm": hbm, "alu": alu}
    rec.update(extra)
    return rec


def measured_traffic(*kernels: str):
    """HBM bytes per launch (summed over the named kernels, which together make one
    launch of the timed unit) from the committed FETCH_SIZE / WRITE_SIZE profile, or None
    when the kernel sources have changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        for rel, want in rec["source_sha256"].items():
            if hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest() != want:
                return None
        return float(sum(rec[k]["bytes_per_launch"] for k in kernels))
    except (OSError, KeyError, ValueError):
        return None


_BARRIER = None


def _cpu_init(barrier):
    global _BARRIER
    _BARRIER = barrier


def _oracle_for(idx):
    from oracle.couette import CouetteOracle
    from paper_1708_05944_amd import workloads
    d = workloads.couette_sweep()[idx]
    return CouetteOracle(R_in=d.R_in, R_out=d.R_out, N_R=d.N_R, ax1=d.ax1, ax2=d.ax2, Kn=d.Kn,
                         tau_model=d.tau_model, u_in=d.u_in, T_in=d.T_in, u_out=d.u_out, T_out=d.T_out)


def _cpu_worker(args):
    """Oracle (plain C FP64, one thread per process) on a list of sweep instances: build
    them (mpmath tables, not timed), wait for every worker, then step each nsteps RK3
    steps from rest; returns (site-velocity updates, wall-clock start, end)."""
    idxs, nsteps = args
    work = []
    for idx in idxs:
        o = _oracle_for(idx)
        work.append((o, o.equilibrium(1.0, 0.0, 0.0, 1.0), o.cfl_dt(0.5)))
    _BARRIER.wait()
    t0 = time.time()
    upd = 0
    for o, F, dt in work:
        o.step(F, dt, nsteps)
        upd += o.NR * o.NV * nsteps
    return upd, t0, time.time()


def host_cores():
    """Host threads this process may use (affinity), capped at 16 (the host CPU share of one
    GPU on the measurement machines), and the CPU model."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(n, 16), os.cpu_count(), model


def cpu_baseline(n_inst: int, nsteps: int, single_inst: int, tts: bool = True):
    """The oracle as it stands, timed on the host by wall clock: all cores (one process per
    core over the first n_inst sweep instances, nsteps steps each, started together
    after their set-up), one thread (the first single_inst instances in turn), and the
    single-instance workload from rest to r < 1e-10 (residual checked every 500 steps)."""
    import multiprocessing as mp
    from oracle import couette as oc
    oc.build()
    cores, nproc, model = host_cores()
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(cores)
    chunks = [(list(range(c, n_inst, cores)), nsteps) for c in range(cores)]
    with ctx.Pool(cores, initializer=_cpu_init, initargs=(barrier,)) as pool:
        res = pool.map(_cpu_worker, chunks, chunksize=1)
    upd = sum(r[0] for r in res)
    wall = max(r[2] for r in res) - min(r[1] for r in res)
    # one thread
    work = []
    for idx in range(single_inst):
        o = _oracle_for(idx)
        work.append((o, o.equilibrium(1.0, 0.0, 0.0, 1.0), o.cfl_dt(0.5)))
    t0 = time.perf_counter()
    upd1 = 0
    for o, F, dt in work:
        o.step(F, dt, nsteps)
        upd1 += o.NR * o.NV * nsteps
    single = upd1 / (time.perf_counter() - t0)
    out = dict(value=upd / wall, unit="site-velocity updates/s", cores=cores, kind="oracle",
               sample=f"sweep instances 0..{n_inst - 1}, {nsteps} RK3 steps each from rest, {cores} processes x 1 "
                      f"thread started together after their table set-up; value = updates / wall-clock "
                      f"({wall:.2f} s)",
               single_thread_value=single,
               single_thread_sample=f"sweep instances 0..{single_inst - 1}, {nsteps} steps each, one thread",
               host={"nproc": nproc, "cpu_model": model})
    if tts:
        from oracle.couette import CouetteOracle
        from paper_1708_05944_amd import workloads
        d = workloads.single_couette()
        o = CouetteOracle(R_in=d.R_in, R_out=d.R_out, N_R=d.N_R, ax1=d.ax1, ax2=d.ax2, Kn=d.Kn,
                          tau_model=d.tau_model, u_in=d.u_in, T_in=d.T_in, u_out=d.u_out, T_out=d.T_out)
        F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
        dt = o.cfl_dt(0.5)
        t0 = time.perf_counter()
        steps, r = 0, float("inf")
        while r >= 1e-10 and steps < 100_000:
            F = o.step(F, dt, 499)
            G = o.step(F, dt, 1)
            r = o.residual(G, F, dt)
            F = G
            steps += 500
        out["time_to_steady_state_single"] = dict(seconds=time.perf_counter() - t0, steps=steps, residual=r, dt=dt,
                                                  converged=bool(r < 1e-10), threads=1)
    return out


def channel_cpu_baseline():
    """The channel oracle (plain C FP64, one thread; a single instance is one serial sweep)
    for one RK3 step of the 512 x 128 channel from rest."""
    import numpy as np
    from oracle.channel import ChannelOracle
    from paper_1708_05944_amd import workloads
    d = workloads.channel_512x128()
    o = ChannelOracle(NL=d.N_lambda, NX=d.N_xi, ax1=d.ax1, ax2=d.ax2, Kn=d.Kn, tau_model=d.tau_model, r=d.r, L=d.L,
                      xi_in=d.xi_in, xi_out=d.xi_out, n_in=d.n_in, n_out=d.n_out, T_w=d.T_w)
    F = o.equilibrium(1.0, 0.0, 0.0, 1.0)
    dt = o.cfl_dt(0.5)
    t0 = time.perf_counter()
    F = o.step(F, dt, 1)
    el = time.perf_counter() - t0
    assert np.isfinite(F).all()
    sv = d.N_lambda * d.N_xi * o.NV
    return dict(value=sv / el, unit="site-velocity updates/s", cores=1, kind="oracle",
                sample=f"one RK3 step of the 512 x 128 channel (256 velocities) from rest, one thread "
                       f"({el:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-instances", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-single", type=int, default=8, help="sweep instances of the single-thread oracle timing")
    ap.add_argument("--no-tts", action="store_true",
                    help="skip the single-instance time-to-steady-state leg (profiling runs)")
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the learned warm-start leg (training solves, training, held-out runs)")
    ap.add_argument("--no-channel", action="store_true", help="skip the expanding-channel leg")
    ap.add_argument("--no-ballistic", action="store_true", help="skip the ballistic (8000-velocity) leg")
    ap.add_argument("--no-channel-sweep", action="store_true", help="skip the batched 64-channel leg")
    ap.add_argument("--no-clb", action="store_true", help="skip the vielbein vs Cartesian-split channel timing")
    ap.add_argument("--warm-train", type=int, default=4096, help="training instances of the warm-start leg")
    ap.add_argument("--warm-heldout", type=int, default=256, help="held-out instances of the warm-start leg")
    ap.add_argument("--warm-epochs", type=int, default=100, help="training epochs of the warm-start leg")
    ap.add_argument("--no-channel-warm", action="store_true", help="skip the learned channel warm-start leg")
    ap.add_argument("--no-eps-free", action="store_true", help="skip the epsilon-free held-out runs of the warm leg")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="after the run, one plain device copy of this many MiB (reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(instances shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1708_05944_amd import VLB_MIXED, Batch, workloads

    descs = workloads.couette_sweep()
    updates_per_step = workloads.site_velocities(descs)

    def measure(precision):
        batch = Batch(descs, precision=precision)
        batch.step(1)                          # moves a mixed batch into its FP32 buffers
        tile, _ = batch.autotune(3)            # cells per run of the stage kernel, by timing
        batch.step(args.warmup)
        torch.cuda.synchronize()
        batch.timing_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        groups = batch.timing_query()
        batch.timing_enable(False)
        r = batch.residual()
        batch.close()
        dom = max(groups, key=lambda g: g["total_ms"])
        return dict(value=updates_per_step * args.steps / el, ms_per_step=el / args.steps * 1e3, dom=dom,
                    max_residual=float(r.max()), tile=tile)

    fp64 = measure(0)
    mixed = measure(VLB_MIXED)
    dom, dom64 = mixed["dom"], fp64["dom"]
    couette_flops_launch = stage_flops(descs)
    roof = roofline("couette_stage<float, false>", dom["total_ms"] / dom["launches"], dom["alg_bytes"] / dom["launches"],
                    couette_flops_launch, VALU_FP32_TFLOPS, measured_traffic("couette_stage<float, false>"),
                    launches=dom["launches"])
    roof64 = roofline("couette_stage<double, false>", dom64["total_ms"] / dom64["launches"],
                      dom64["alg_bytes"] / dom64["launches"], couette_flops_launch, VALU_FP64_TFLOPS,
                      measured_traffic("couette_stage<double, false>"), launches=dom64["launches"])

    # time to steady state (r < 1e-10) of the single-instance workload, FP64 vs mixed
    tts = {}
    for name, prec in (() if args.no_tts else (("fp64", 0), ("mixed", VLB_MIXED))):
        b = Batch([workloads.single_couette()], precision=prec)
        b.step(0 if prec == 0 else 1)
        single_tile, _ = b.autotune(20)
        b.init_equilibrium(0, 1.0, 0.0, 0.0, 1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, r, ok = b.run_to_steady(1e-10, 100000, 500)
        torch.cuda.synchronize()
        tts[name] = dict(seconds=time.perf_counter() - t0, steps=int(steps[0]), converged=bool(ok),
                         fp32_steps=int(b.mixed_report()[2][0]) if prec else 0, tile=single_tile)
        b.close()

    channel = None
    if not args.no_channel:
        # expanding channel, 512 x 128 cells, HH(4;8) x H(4;16) = 256 velocities, Kn = 0.05,
        # pressure-driven (n 1.1 -> 0.9), expansion ratio 2 over 4 widths; mixed precision
        # (FP32 stage kernel with FP32 MFMA contractions, FP64 sums) and FP64
        from paper_1708_05944_amd import Channel, ChannelDesc
        cd = ChannelDesc(N_lambda=128, N_xi=512, xi_in=-4.0, xi_out=12.0, r=2.0, L=4.0, ax1=(1, 8, 4),
                         ax2=(0, 16, 4), Kn=0.05, tau_model=1, n_in=1.1, n_out=0.9, T_w=1.0)
        sv = cd.N_lambda * cd.N_xi * 16 * 16
        ch_flops_launch = channel_stage_flops(cd.N_lambda * cd.N_xi, 16, 16)

        def channel_leg(precision, elem_bytes, tname, peak_tf):
            # one RK3 stage = the interior launch and the edge-band launch
            kernels = [f"channel_stage<{tname}, 1, 1, {b}>" for b in ("false", "true")]
            ch = Channel([cd], precision=precision)
            ch.step(2)
            torch.cuda.synchronize()
            nst = max(2, args.steps // 2)
            # HIP events on the stream the library launches on (the current torch stream):
            # the nst steps are 3 nst stages (an interior and an edge-band launch each) plus one
            # residual reduction (~0.15 ms)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record()
            ch.step(nst)
            e1.record()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            stage_ms = e0.elapsed_time(e1) / (3 * nst)
            dt = ch.info[0]["dt"]
            ch.close()
            bytes_launch = sv * 16 * elem_bytes / 3      # read F, F_n in 2 of 3 stages, write
            return {"value": sv * nst / el, "unit": "site-velocity updates/s", "ms_per_step": el / nst * 1e3,
                    "steps": nst, "dt": dt,
                    "roofline": roofline(" + ".join(kernels), stage_ms, bytes_launch, ch_flops_launch, peak_tf,
                                         measured_traffic(*kernels))}

        mixed_ch = channel_leg(VLB_MIXED, 4, "float", VALU_FP32_TFLOPS)
        fp64_ch = channel_leg(0, 8, "double", VALU_FP64_TFLOPS)
        channel = {"workload": "expanding channel 512 x 128 cells, HH(4;8) x H(4;16) (256 velocities), Kn 0.05, "
                               "ratio 2 over 4 widths, reservoirs n 1.1 / 0.9; mixed = FP32 stage kernel on "
                               "weight-scaled populations with FP32 MFMA contractions and FP64 sums",
                   **mixed_ch, "dtype": "f32", "fp64": fp64_ch}

    channel_batch = None
    if not args.no_channel_sweep:
        # batched expanding channels: 64 seeded instances (N_lambda 64..256, N_xi = 4 N_lambda,
        # Kn 0.01..1, expansion ratio 1.5..3, HH(4;Q) x H(4;16) with Q 8..16 by Kn: 256..512
        # velocities, both velocity-tile classes), advanced together; HIP events around the
        # timed steps (graph-replayed stages of every instance)
        from paper_1708_05944_amd import Channel
        sweep = workloads.channel_sweep()
        sv_b = sum(d.N_lambda * d.N_xi * 2 * d.ax1[1] * d.ax2[1] for d in sweep)

        def batch_leg(precision):
            torch.cuda.empty_cache()   # the batch takes 134 GB (FP64) / 201 GB (mixed) of HBM
            c = Channel(sweep, precision=precision)
            c.step(1)
            torch.cuda.synchronize()
            nst = 3
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            c.step(nst)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / nst
            c.close()
            return {"value": sv_b / (ms * 1e-3), "unit": "site-velocity updates/s", "ms_per_step": ms, "steps": nst}

        channel_batch = {"workload": "64 expanding channels (PCG64 seed 3): N_lambda 64-256 x N_xi 4 N_lambda, "
                                     "Kn 0.01-1, ratio 1.5-3 over 4 widths, HH(4;8..16) x H(4;16) (256-512 "
                                     "velocities), reservoirs n 1.1 / 0.9, one batch",
                         "site_velocities_per_step": sv_b, **batch_leg(VLB_MIXED), "dtype": "f32",
                         "fp64": batch_leg(0)}

    ballistic = None
    if not args.no_ballistic:
        # ballistic regime of the free-molecular comparison: one instance, 16 stretched
        # cells, HH(4;200) x HH(4;10) = 8000 velocities, FP64 on the large-velocity-set
        # stage (K1 F product on the matrix cores, then the per-population update)
        from paper_1708_05944_amd import Batch, CouetteDesc
        bd = CouetteDesc(R_in=1.0, R_out=2.0, N_R=16, ax1=(1, 200, 4), ax2=(1, 10, 4), Kn=1e8, u_in=1.0, A=0.95,
                         delta=0.75)
        bb = Batch([bd])
        bb.step(12)
        torch.cuda.synchronize()
        nst = max(100, 10 * args.steps)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        bb.step(nst)
        e1.record()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        stage_ms = e0.elapsed_time(e1) / (3 * nst)
        n1, n2, NR = 400, 20, 16
        prod_flops = 2.0 * (2 * NR) * n1 * n1 * n2          # K1 F for both distributions, per stage
        ballistic = {"workload": "ballistic circular Couette (Kn 1e8), R 1 -> 2, wall speed 1, 16 cells stretched "
                                 "A 0.95 / delta 0.75, HH(4;200) x HH(4;10) = 8000 velocities, FP64",
                     "value": NR * n1 * n2 * nst / el, "unit": "site-velocity updates/s",
                     "ms_per_step": el / nst * 1e3, "steps": nst, "dt": bb.info[0]["dt"],
                     "stage_ms": stage_ms,
                     "product_TFLOPs_over_stage": prod_flops / (stage_ms * 1e-3) / 1e12,
                     "product_flops_per_stage": prod_flops}
        bb.close()

    clb = None
    if not args.no_clb:
        # vielbein (HH(N;Q) x H(4;5)) against Cartesian-split (HH(N;Q) x HH(N;Q)) channels on the
        # same grid -- 30 x 200 as in the paper's performance comparison of Sec. VI.G, and the
        # 128 x 512 grid that fills the chip -- FP64, each at
        # its own stable dt (the work per step does not depend on it)
        from paper_1708_05944_amd import Channel, ChannelDesc
        rows = []
        for NL, NX, Q in ((30, 200, 4), (30, 200, 8), (30, 200, 12), (30, 200, 16), (128, 512, 8), (128, 512, 16)):
            geo = dict(N_lambda=NL, N_xi=NX, xi_in=-10.0, xi_out=40.0, r=2.0, L=16.0, Kn=0.2, tau_model=1,
                       n_in=1.05, n_out=0.95, T_w=1.0)
            times = {}
            N = min(Q - 1, 4)
            for name, kw in (("vlb", dict(ax1=(1, Q, N), ax2=(0, 5, 4))),
                             ("vlb_pop", dict(ax1=(1, Q, N), ax2=(0, 5, 4), kernel=2)),
                             ("clb", dict(ax1=(1, Q, N), ax2=(1, Q, N), cartesian=True))):
                ch = Channel([ChannelDesc(**geo, **kw)])
                ch.step(2)
                torch.cuda.synchronize()
                nst = 20
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                ch.step(nst)
                e1.record()
                torch.cuda.synchronize()
                times[name] = (e0.elapsed_time(e1) / nst, ch.info[0]["NV"])
                ch.close()
            rows.append({"grid": f"{NL} x {NX}", "Q": Q, "vlb_ms_per_step": times["vlb"][0],
                         "vlb_velocities": times["vlb"][1], "vlb_population_kernel_ms_per_step": times["vlb_pop"][0],
                         "clb_ms_per_step": times["clb"][0], "clb_velocities": times["clb"][1],
                         "time_ratio_vlb_over_clb": times["vlb"][0] / times["clb"][0]})
        clb = {"workload": "expanding channel 30 x 200 (the paper's grid) and 128 x 512 cells (r 2, L 16, "
                           "xi -10..40), Kn 0.2, FP64; vielbein "
                           "HH(N;Q) x H(4;5) (16 x 16 velocity tiles, the automatic choice; also on the population "
                           "kernel) vs Cartesian-split HH(N;Q) x HH(N;Q), N = min(Q - 1, 4); ms per RK3 step "
                           "(HIP events)",
               "rows": rows}

    warm = None
    if not args.no_warm:
        # learned warm start: surrogate trained on the solver's own steady states (sweep
        # generator, seed 1), evaluated on held-out instances (seed 2), cold and warm, in FP64
        # and by the mixed defect correction; family Kn <= 0.2, 32 cells; the regularised WENO
        # weights (1e-6) give every instance of the family a steady state, and the held-out set
        # is also run with the paper's epsilon-free weights
        from paper_1708_05944_amd import surrogate
        log = lambda m: print(m, file=sys.stderr, flush=True)
        tr = workloads.surrogate_descs(args.warm_train, workloads.SURROGATE_TRAIN_SEED, N_R=32, Kn_max=0.2)
        ho = workloads.surrogate_descs(args.warm_heldout, workloads.SURROGATE_HELDOUT_SEED, N_R=32, Kn_max=0.2)
        for d in tr + ho:
            d.weno_eps = 1e-6
        ho0 = workloads.surrogate_descs(args.warm_heldout, workloads.SURROGATE_HELDOUT_SEED, N_R=32, Kn_max=0.2)
        log(f"warm start: {len(tr)} training solves")
        warm = surrogate.warm_start_comparison(tr, ho, epochs=args.warm_epochs, batch=256, lr=1e-3, probe=500,
                                               max_steps=200_000, chunk=10_000, log=log,
                                               extra=None if args.no_eps_free else {"epsilon_free": ho0})
        warm["workload"] = (f"learned warm start, weno_eps 1e-6: {len(tr)} training / {len(ho)} held-out Couette "
                            f"instances of the sweep generator (seeds 1 / 2) restricted to Kn <= 0.2 and 32 cells; "
                            f"cold = rest state, warm = surrogate (bf16 inference) + 500-step FP64 acceptance probe "
                            f"+ stall watch (cold restart after 10000 steps without a new residual low); each in FP64 "
                            f"and in mixed precision (defect correction); non-converged instances count the whole "
                            f"200000-step budget; 'extra.epsilon_free': the same held-out instances with the paper's "
                            f"epsilon-free WENO weights, warm-started by the same network")
        log("warm start done")

    channel_warm = None
    if not args.no_channel_warm:
        # learned warm start of batched expanding channels: a reduced channel family (32 x 8
        # cells, 64 velocities, Kn 0.04-0.25, r 1.5-3) whose members all reach r < 1e-10;
        # surrogate trained on 32 channel steady states (seed 11), 16 held-out channels
        # (seed 12) run cold and warm in FP64
        from paper_1708_05944_amd import surrogate
        log = lambda m: print(m, file=sys.stderr, flush=True)
        tr = workloads.channel_surrogate_descs(32, workloads.CHANNEL_SURROGATE_TRAIN_SEED)
        ho = workloads.channel_surrogate_descs(16, workloads.CHANNEL_SURROGATE_HELDOUT_SEED)
        log("channel warm start: 32 training solves")
        channel_warm = surrogate.channel_warm_comparison(tr, ho, epochs=300, max_steps=200_000, log=log)
        channel_warm["workload"] = ("learned warm start of expanding channels: 32 training / 16 held-out channels "
                                    "(seeds 11 / 12), 32 x 8 cells, HH(3;4) x H(4;8), Kn log-uniform 0.04-0.25 "
                                    "(tau = Kn/(nT)), r uniform 1.5-3 over L = 4, reservoirs 1.1 / 0.9, weno_eps "
                                    "1e-6; inputs (log Kn, r, xi, lambda); cold = rest state, warm = local "
                                    "equilibrium of the surrogate's fields (bf16 inference) + stall watch (cold "
                                    "restart after 40000 steps without a new residual low); FP64 to r < 1e-10; "
                                    "non-converged instances count the whole 200000-step budget")
        log("channel warm start done")

    out = {
        "metric": "site-velocity updates/s (batched Couette sweep, mixed precision: FP32 streaming)",
        "value": mixed["value"],
        "unit": "site-velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched circular-Couette sweep: 256 seeded instances (PCG64 seed 20261203), "
                               "64-512 cells, HH(N;4..16) x H(N;4..20) velocity sets (32-640 velocities), "
                               "Kn 0.01-10; FP32 stage kernels with FP64 moment/wall/residual sums",
                   "instances": len(descs), "site_velocities_per_step": updates_per_step,
                   "cells_per_run": mixed["tile"]},
        "roofline": roof,
        "fp64": {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"], "cells_per_run": fp64["tile"],
                 "roofline": roof64},
        "time_to_steady_state_single": tts,
        "time_to_steady_state_warm_start": warm,
        "time_to_steady_state_channel_warm_start": channel_warm,
        "channel": channel,
        "channel_batch": channel_batch,
        "ballistic": ballistic,
        "vlb_vs_clb": clb,
    }
    if args.copy_ref_mib:
        n = args.copy_ref_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_ref_bytes"] = n
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_instances, args.cpu_steps, args.cpu_single, tts=not args.no_tts)
        if channel is not None:
            channel["cpu_baseline"] = channel_cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
