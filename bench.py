#!/usr/bin/env python3
"""Throughput of the chi(2) split-step z-loop on one MI355X.

A "step" is one z-step of the method (RK4 half-step, forward transforms,
propagator, inverse transforms, RK4 half-step) over the whole grid.  The
timed workload is the 3-field OPG solve on a 256^3 grid (about 400 MB of
complex64 state, larger than the 256 MB last-level cache), seeded synthetic
input, fields resident in HBM before timing starts.

Prints one JSON line: grid-point z-steps per second, the HBM roofline of the
whole z-step (its passes' algorithmic bytes over their event-timed
durations, with every pass kind and the dominant kernel listed beside it),
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-point·z-steps/s + % HBM peak; adjoint/forward time; batched vs plain"
HBM_PEAK_GBS = 8000.0
# MI355X FP32 vector peak (published, with packed FP32 math) and the peak of
# the unpacked FP32 instructions these kernels are built with: 256 CUs x 4
# SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed z-steps (1000 = full solve)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="opg256", choices=["opg256", "sfg128", "shg32"])
    ap.add_argument("--timing-steps", type=int, default=200,
                    help="z-steps of the event-timed run used for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint and batched-sweep side measurements")
    ap.add_argument("--extras", default="all",
                    help="comma-separated side measurements to run (adjoint, batch, reduced_dims, "
                         "diagnostics, dk_map, paper_grids) or 'all'")
    ap.add_argument("--cpu-steps", type=int, default=4, help="oracle z-steps in the CPU sample")
    ap.add_argument("--pass-order", default="auto", choices=["auto", "0", "1", "2", "3"],
                    help="plan schedule: autotuned (default) or a fixed pass order")
    ap.add_argument("--wide", type=int, default=0,
                    help="with a fixed pass order: axes (bits x=1, y=2, tau=4) whose linear passes "
                         "run 512-thread blocks")
    ap.add_argument("--literal-halves", action="store_true",
                    help="keep both RK4 half-steps of every step (no merging of adjacent halves)")
    ap.add_argument("--no-fuse", action="store_true",
                    help="with a fixed pass order: three passes per step (no fused step pairs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time a plain 1 GiB device-to-device copy instead (reference for "
                         "achievable bandwidth and for scaling hardware byte counters)")
    return ap.parse_args()


def copy_calibration():
    """Plain device copy of a known size: 2 x 1 GiB of HBM traffic per copy."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    reps = 10
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "avg_ms": ms,
                      "GBps_read_plus_write": 2 * n / (ms * 1e-3) / 1e9}), flush=True)


def adjoint_ratio(dev, reps=3):
    """Inverse-design workload (SHG 128x128x64, 400 steps, per-step dk profile,
    checkpoints every 20 steps): time of (forward with checkpoints + reverse
    sweep) over the time of a plain forward solve, medians of `reps` runs."""
    import torch
    from paper_2609_08384_amd import brahms, inputs
    wl = inputs.shg_adjoint()
    params = brahms.params_from_workload(wl)
    init = [torch.from_numpy(a).to(dev) for a in wl.init]

    def run(adjoint):
        fields = [a.clone() for a in init]
        plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, params).bind(fields)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if adjoint:
            plan.adjoint_forward(wl.nz, 20)
            g = [torch.zeros_like(f) for f in fields]
            g[1].copy_(-2 * fields[1])      # J = -sum |S(L)|^2
            plan.adjoint_backward(g)
        else:
            plan.step(wl.nz)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plan.destroy()
        return dt

    run(False)
    run(True)
    fwd = sorted(run(False) for _ in range(reps))[reps // 2]
    adj = sorted(run(True) for _ in range(reps))[reps // 2]
    return {"workload": f"{wl.name}: SHG {wl.nx}x{wl.ny}x{wl.nt}, {wl.nz} z-steps, per-step dk, "
                        "checkpoint every 20 steps",
            "forward_ms": fwd * 1e3, "forward_plus_adjoint_ms": adj * 1e3, "ratio": adj / fwd}


def _median_time(fn, reps=3):
    fn()
    return sorted(fn() for _ in range(reps))[reps // 2]


def reduced_dims(dev):
    """Focusing sweep of 99 CW problems (128 x 128 x 1, 200 steps each; the
    Boyd-Kleinman study of Sec. 5.2) as one batch, against the same problems
    propagated one after another with plain plans (both with merged RK4
    half-steps)."""
    import torch
    from paper_2609_08384_amd import brahms, inputs
    wls = inputs.bk_sweep()
    init = [[torch.from_numpy(a).to(dev) for a in w.init] for w in wls]
    fields = [[a.clone() for a in fs] for fs in init]
    batch = brahms.Batch([(w.nx, w.ny, w.nt, w.nf, brahms.params_from_workload(w), w.nz) for w in wls])
    batch.set_merge_halves(1)
    batch.bind(fields)

    def run_batch():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.run()
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    t_batch = _median_time(run_batch)
    batch.destroy()
    plans = []
    for w, fs in zip(wls, fields):
        pl = brahms.Plan(w.nx, w.ny, w.nt, w.nf, brahms.params_from_workload(w))
        pl.set_schedule(0, 0, 1)
        plans.append(pl.bind(fs))

    def run_seq():
        for pl in plans:
            pl.set_z(0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pl, w in zip(plans, wls):
            pl.step(w.nz)
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    t_seq = _median_time(run_seq)
    for pl in plans:
        pl.destroy()
    work = sum(w.points * w.nz for w in wls)
    return {"workload": "99 CW SHG problems 128x128x1 (xi 2..4 x dk L -4..-2.4), 200 steps",
            "batched_ms": t_batch * 1e3, "sequential_ms": t_seq * 1e3, "speedup": t_seq / t_batch,
            "batched_rate": work / t_batch}


def diagnostics_cost(dev, wl, steps=100, every=10):
    """One diagnostics record of the benchmark grid (event-timed, bytes read
    = 8 nf per point) and the cost of recording every `every` steps."""
    import torch
    from paper_2609_08384_amd import brahms
    fields = [torch.from_numpy(a).to(dev) for a in wl.init]
    plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, brahms.params_from_workload(wl)).bind(fields)
    rec = torch.empty(plan.record_size(), dtype=torch.float64, device=dev)
    plan.diagnose_into(rec)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        plan.diagnose_into(rec)
    ev1.record()
    torch.cuda.synchronize()
    rec_ms = ev0.elapsed_time(ev1) / 10

    def run(monitor):
        plan.set_z(0.0)
        plan.set_monitor(every if monitor else 0, steps // every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    plain = _median_time(lambda: run(False))
    mon = _median_time(lambda: run(True))
    plan.destroy()
    nbytes = 8 * wl.nf * wl.points
    return {"record_ms": rec_ms, "record_GBps": nbytes / (rec_ms * 1e-3) / 1e9,
            "steps": steps, "every": every, "plain_ms": plain * 1e3, "monitored_ms": mon * 1e3,
            "overhead": mon / plain - 1.0}


def dk_map_cost(dev):
    """SHG 128 x 128 x 64 with a transverse mismatch map (200 steps) against
    the same problem without the map."""
    import torch
    from paper_2609_08384_amd import brahms, inputs
    wl = inputs.shg_thermal()
    out = {}
    for name, with_map in (("with_map_ms", True), ("without_map_ms", False)):
        prm = brahms.params_from_workload(wl)
        if not with_map:
            prm.dk_map, prm.dk_map_scale = None, None
        fields = [torch.from_numpy(a).to(dev) for a in wl.init]
        plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, prm).bind(fields)

        def run():
            plan.set_z(0.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.step(wl.nz)
            torch.cuda.synchronize()
            return time.perf_counter() - t0
        out[name] = _median_time(run) * 1e3
        plan.destroy()
    out["workload"] = "shg_thermal: SHG 128x128x64, 200 steps, transverse dk map"
    out["overhead"] = out["with_map_ms"] / out["without_map_ms"] - 1.0
    return out


# (grid, paper's GPU-3 time in s for 100 000 steps, tab. gpu_runtime):
# context only, other hardware, FP32, a physical MgO:PPLN workload
PAPER_GRIDS = [((64, 64, 4096), 16611.0), ((128, 128, 1024), 5141.0)]


def paper_grids(dev, steps=200):
    """Three-field pulsed-focused grids of the paper's runtime table on this
    engine: seeded OPG-type fields, `steps` timed steps after a warm-up."""
    import numpy as np
    import torch
    from paper_2609_08384_amd import autotune, brahms, inputs
    out = []
    for (nx, ny, nt), paper_s in PAPER_GRIDS:
        fs = [inputs.FieldSpec(kappa=2.0 * w, diffraction=20.0 / w, tan_rho=1.0, delay=10.0 * j,
                               k2=500.0 * (1 - j)) for j, w in enumerate(inputs.OMEGA_RATIO)]
        params = brahms.Params(dz=1e-3, fields=[brahms.FieldParams(f.kappa, f.diffraction, f.tan_rho,
                                                                   f.delay, f.k2) for f in fs])
        pump = inputs.focused_pulse(nx, ny, nt, nx / 8.0, inputs.fwhm_to_tau0(nt / 8.0), 0.5)
        rng = np.random.default_rng(nt)
        seeds = [1e-6 * (rng.standard_normal((nt, ny, nx)) + 1j * rng.standard_normal((nt, ny, nx)))
                 for _ in range(2)]
        fields = [torch.from_numpy(inputs.to_c64(a)).to(dev) for a in [pump] + seeds]
        plan = brahms.Plan(nx, ny, nt, 3, params).bind(fields)
        sched = autotune.apply(plan, dev)
        plan.step(64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plan.destroy()
        n = nx * ny * nt
        rate = n * steps / dt
        out.append({"grid": f"{nx}x{ny}x{nt}", "fields": 3, "ms_per_step": dt / steps * 1e3,
                    "rate": rate, "hbm_frac_step": (5 if nt > 256 else 3) * 48 * n / (dt / steps) / 8e12,
                    "schedule": sched, "paper_gpu3_rate": n * 1e5 / paper_s,
                    "vs_paper_gpu3": rate / (n * 1e5 / paper_s)})
    return out


def batch_ratio(dev):
    """Seeded SHG sweep (64 problems over 64^3, 96x96x64, 128x128x64 and
    128x128x256 grids, dk L in [-6, 6], xi in [0.1, 10], 200-600 steps): one
    batched run (autotuned: one hipGraph, or its launch groups on several
    streams) against the same 64 problems propagated one after another with
    plain plans (each with its shape's tuned schedule, no synchronisation
    between them); medians of 3."""
    import torch
    from paper_2609_08384_amd import autotune, brahms, inputs
    wls = inputs.shg_sweep(seed=4, count=64)
    probs = [(w.nx, w.ny, w.nt, w.nf, brahms.params_from_workload(w), w.nz) for w in wls]
    init = [[torch.from_numpy(a).to(dev) for a in w.init] for w in wls]
    fields = [[a.clone() for a in fs] for fs in init]

    def reset():
        for fs, gs in zip(fields, init):
            for f, g in zip(fs, gs):
                f.copy_(g)
        torch.cuda.synchronize()

    batch = brahms.Batch(probs)
    # the tuner's six fastest probe candidates re-timed over whole runs of
    # the sweep (fields restored after)
    tuned = autotune.tune_batch(batch, dev, run_fields=fields)
    batch.bind(fields)
    batch.run()                      # builds the graph

    def run_batch():
        reset()
        t0 = time.perf_counter()
        batch.run()
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    t_batch = sorted(run_batch() for _ in range(3))[1]
    groups = batch.groups()
    batch.destroy()

    # the sequential solves each take the order that is fastest for a plain
    # solve of their shape
    plans = []
    for w, fs in zip(wls, fields):
        pl = brahms.Plan(w.nx, w.ny, w.nt, w.nf, brahms.params_from_workload(w))
        autotune.apply(pl, dev)
        plans.append(pl.bind(fs))
    for pl in plans:                 # first launches of every kernel variant
        pl.step(2)
        pl.set_z(0.0)
    def run_seq():
        for pl in plans:
            pl.set_z(0.0)
        reset()
        t0 = time.perf_counter()
        for pl, w in zip(plans, wls):
            pl.propagate(w.nz * w.dz)
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    t_seq = sorted(run_seq() for _ in range(3))[1]
    for pl in plans:
        pl.destroy()
    work = sum(w.points * w.nz for w in wls)
    return {"workload": "SHG sweep: 64 problems, grids 64^3 / 96x96x64 / 128x128x64 / 128x128x256, "
                        "200-600 steps (seed 4)",
            "grid_point_steps": work, "batched_ms": t_batch * 1e3, "sequential_ms": t_seq * 1e3,
            "speedup": t_seq / t_batch, "batched_rate": work / t_batch,
            "sequential_rate": work / t_seq, "launch_groups": groups,
            "schedule": tuned["choice"], "group_max": tuned["group_max"], "streams": list(tuned["streams"]), "wide": tuned.get("wide"),
            "group_limits": tuned["group_limits"], "batch_orders": tuned["orders"],
            "tuner_probe_ms": tuned["probe_ms"], "tuner_shape_probe_ms": tuned["shape_probe_ms"],
            "tuner_whole_run_ms": tuned["whole_run_ms"]}


# Sources that define the pass kernels and their launch configuration: the
# HBM byte counts recorded under profiles/ hold only for the digest of these.
KERNEL_SOURCES = ("paper_2609_08384_amd/csrc/kernels.hpp", "paper_2609_08384_amd/csrc/dft.hpp",
                  "paper_2609_08384_amd/csrc/lengths.hpp", "paper_2609_08384_amd/csrc/launch_impl.hpp",
                  "paper_2609_08384_amd/csrc/len_256.hip", "paper_2609_08384_amd/csrc/engine.hip")
NL_OF_PASS = {0: {"x_pass": "before", "y_pass": "none", "t_pass": "after"},
              1: {"t_pass": "before", "y_pass": "none", "x_pass": "after"},
              2: {"x_pass": "before", "t_pass": "none", "y_pass": "after"},
              3: {"y_pass": "before", "t_pass": "none", "x_pass": "after"}}


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def nl_of_pass(pass_order: int, merge_halves: int, fuse_steps: int = 0) -> dict:
    """RK4 mode of each pass in the steady state of a run: with merged
    half-steps the first pass of every step but the run's first is linear;
    with fused step pairs the first and last axes alternate as the pass that
    ends one step and begins the next ("fused")."""
    modes = dict(NL_OF_PASS[pass_order])
    if merge_halves and fuse_steps:
        return {k: ("none" if v == "none" else "fused") for k, v in modes.items()}
    if merge_halves:
        modes = {k: ("none" if v == "before" else v) for k, v in modes.items()}
    return modes


def fused_pass_flops(nf: int, points: int, n_axis: int) -> float:
    """Algorithmic FP32 flops of one fused pass: per grid point and field two
    round trips along the axis (forward and inverse transform at the
    conventional 5 N log2 N flops each, and the 6-flop propagator product)
    and one RK4 step of the coupled equations (per field four stages of one
    complex product of two fields, 6 flops, the product with the stage
    coefficient, 6, the stage update, 2, and the weighted accumulation, 8)."""
    import math
    per_trip = 2 * 5 * math.log2(n_axis) + 6
    return float(points) * nf * (2 * per_trip + 4 * (6 + 6 + 2 + 8))


def measured_traffic(workload: str, pass_name: str, pass_order: int, merge_halves: int = 0,
                     fuse_steps: int = 0, wide: int = 0):
    """HBM bytes per launch of one pass kernel from the hardware-counter
    summary profiles/hbm_traffic_<workload>.json (FETCH_SIZE and WRITE_SIZE
    per dispatch, each scaled by what the counter reads for a plain copy of
    known size), or None when there is no summary for this kernel or the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_digest") != kernel_digest():
        return None
    mode = nl_of_pass(pass_order, merge_halves, fuse_steps)[pass_name]
    axis_bit = {"x_pass": 1, "y_pass": 2, "t_pass": 4}[pass_name]
    # linear passes on 512-thread blocks are kernels of their own
    key = f"{pass_name}:{mode}" + (":wide" if mode == "none" and wide & axis_bit else "")
    k = rec.get("kernels", {}).get(key)
    if k is None:
        return None
    return int(round(k["fetch_kib"] * 1024 * rec["fetch_factor"] + k["write_kib"] * 1024 * rec["write_factor"]))


def make_workload(name):
    from paper_2609_08384_amd import inputs
    return {"opg256": inputs.opg256, "sfg128": inputs.sfg128, "shg32": inputs.shg32}[name]()


def cpu_baseline(wl, nsteps):
    """The FP64 oracle (test infrastructure) on the first nsteps z-steps of
    the same workload, on this host's cores."""
    import torch
    from oracle import ssfm
    fields = [ssfm.FieldParams(kappa=f.kappa, diffraction=f.diffraction, tan_rho=f.tan_rho,
                               delay=f.delay, k2=f.k2, k3=f.k3, alpha=f.alpha) for f in wl.fields]
    prob = ssfm.Problem(wl.nx, wl.ny, wl.nt, wl.nf, wl.dz, fields, dk_const=wl.dk_const,
                        dk=None if wl.dk is None else list(wl.dk))
    orc = ssfm.Oracle(prob)
    a = [torch.from_numpy(x).to(torch.complex128) for x in wl.init]
    a = orc.step(a, 0)  # first step outside the clock (allocator warm-up)
    t0 = time.perf_counter()
    for n in range(1, 1 + nsteps):
        a = orc.step(a, n)
    dt = time.perf_counter() - t0
    return {"value": wl.points * nsteps / dt, "unit": "grid-point·z-steps/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{wl.name}: {nsteps} z-steps of the full {wl.nx}x{wl.ny}x{wl.nt} grid, "
                      f"{wl.nf} fields, complex128, {dt:.1f} s",
            "cpu": cpu_model(), "os_cores": os.cpu_count()}


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), or what platform reports."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: only one GPU is supported (asked for {max(args.gpus, world)}); "
              "the engine has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    import numpy as np
    import torch
    from paper_2609_08384_amd import brahms

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = make_workload(args.workload)
    init = [torch.from_numpy(a).to(dev) for a in wl.init]
    fields = [a.clone() for a in init]
    plan = brahms.Plan(wl.nx, wl.ny, wl.nt, wl.nf, brahms.params_from_workload(wl)).bind(fields)
    if args.pass_order == "auto":
        from paper_2609_08384_amd import autotune
        schedule = autotune.apply(plan, dev, merge_halves=not args.literal_halves)
    else:
        merge = 0 if args.literal_halves else 1
        plan.set_schedule(int(args.pass_order), 0, merge, merge and not args.no_fuse, 0, args.wide)
        schedule = plan.get_schedule()

    def reset():
        for f, a in zip(fields, init):
            f.copy_(a)
        plan.set_z(0.0)
        torch.cuda.synchronize()

    # warm-up, then restart the solve from the entrance face
    plan.step(args.warmup)
    reset()

    steps = args.steps
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    plan.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    value = wl.points * steps / wall

    finite = all(bool(torch.isfinite(torch.view_as_real(f)).all()) for f in fields)

    # event-timed run of the same solve for per-kernel durations
    reset()
    plan.timing_enable(True)
    tsteps = min(args.timing_steps, steps)
    plan.step(tsteps)
    tim = plan.timing_read()
    plan.timing_enable(False)
    passes = {k: v for k, v in tim.items() if k != "tables"}
    # algorithmic bytes of one pass launch: every field read once and written
    # once, 2 * 8 B per complex64 value
    bytes_per_launch = 2 * 8 * wl.nf * wl.points
    order, merge, fuse = (int(schedule["pass_order"]), int(schedule.get("merge_halves", 0)),
                          int(schedule.get("fuse_steps", 0)))
    modes = nl_of_pass(order, merge, fuse)
    per_kernel = {k: {"avg_ms": round(v[0] / max(v[1], 1), 5), "launches": v[1],
                      "GBps": (round(bytes_per_launch / (v[0] / v[1] * 1e-3) / 1e9, 1)
                               if v[1] and k != "tables" else None)} for k, v in tim.items()}
    for k, rec in per_kernel.items():
        if k in modes:
            rec["rk4"] = modes[k]
            if modes[k] == "fused" and rec["launches"]:
                n_axis = {"x_pass": wl.nx, "y_pass": wl.ny, "t_pass": wl.nt}[k]
                tf = fused_pass_flops(wl.nf, wl.points, n_axis) / (rec["avg_ms"] * 1e-3) / 1e12
                rec.update({"bound": "alu", "TFLOPs": round(tf, 2), "frac": round(tf / FP32_PEAK_TFLOPS, 4),
                            "frac_of_unpacked_fp32_peak": round(tf / FP32_UNPACKED_TFLOPS, 4),
                            "hbm_frac": round(rec["GBps"] / HBM_PEAK_GBS, 4)})
            elif rec["GBps"]:
                rec.update({"bound": "hbm", "frac": round(rec["GBps"] / HBM_PEAK_GBS, 4)})
    # the dominant kernel: the pass kind with the largest share of the step
    # time, the fused passes of the two alternating axes counted as one kind
    kinds = {}
    for k, (ms, n) in passes.items():
        kind = "fused_pass" if modes.get(k) == "fused" else k
        t = kinds.setdefault(kind, [0.0, 0, []])
        t[0] += ms
        t[1] += n
        t[2].append(k)
    dom = max(kinds, key=lambda k: kinds[k][0])
    dom_ms, dom_n, dom_members = kinds[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    if dom == "fused_pass":
        axis_len = {"x_pass": wl.nx, "y_pass": wl.ny, "t_pass": wl.nt}[dom_members[0]]
        flops = fused_pass_flops(wl.nf, wl.points, axis_len)
        tflops = flops / (avg_ms * 1e-3) / 1e12
        dominant = {"kernel": dom, "axes": dom_members, "bound": "alu", "achieved": round(tflops, 2),
                    "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tflops / FP32_PEAK_TFLOPS, 4),
                    "frac_of_unpacked_fp32_peak": round(tflops / FP32_UNPACKED_TFLOPS, 4),
                    "hbm_GBps": round(achieved, 1), "algorithmic_flops_per_launch": flops,
                    "avg_launch_ms": round(avg_ms, 5), "share_of_step_time": round(dom_ms / sum(
                        v[0] for v in passes.values()), 4)}
    else:
        dominant = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg_ms, 5)}
    # the whole z-step against the HBM roofline: the passes of one step each
    # read and write every field once (the design's pass model, 16 nf P bytes
    # per grid point with P passes per step), timed by the HIP events around
    # the timed region (so launch gaps count), with the summed pass durations
    # of the event-timed run beside it
    long_t = wl.nt > 256
    p_step = (4 if long_t else 2) if (merge and fuse) else (5 if long_t else 3)
    step_bytes = p_step * bytes_per_launch
    timed_steps = max(1, tsteps)
    summed_ms = sum(v[0] for v in tim.values()) / timed_steps
    step_ms = ev_ms / steps
    step_gbs = step_bytes / (step_ms * 1e-3) / 1e9
    traffic = None
    pass_traffic = {k: measured_traffic(wl.name, k, order, merge, fuse, int(schedule.get("wide", 0)))
                    for k in passes if passes[k][1]}
    if pass_traffic and all(v is not None for v in pass_traffic.values()):
        # launches per step of each pass kind in the steady state
        traffic = int(round(sum(pass_traffic[k] * passes[k][1] for k in pass_traffic) / timed_steps))
    roofline = {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(step_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"whole z-step ({p_step} pass launches)", "unit_of_work": "one z-step",
                "algorithmic_bytes_per_step": step_bytes, "step_ms_event": round(step_ms, 5),
                "step_ms_summed_pass_durations": round(summed_ms, 5),
                "passes": {k: {kk: vv for kk, vv in per_kernel[k].items()} for k in passes},
                "dominant_kernel": dominant}
    bytes_per_pt = {"pass_model": 16 * wl.nf * p_step, "compulsory": 16 * wl.nf,
                    "measured": None if traffic is None else round(traffic / wl.points, 3)}
    if traffic is not None:
        bytes_per_pt["measured_over_pass_model"] = round(traffic / wl.points / (16 * wl.nf * p_step), 4)
        bytes_per_pt["measured_over_compulsory"] = round(traffic / wl.points / (16 * wl.nf), 4)
    plan.destroy()

    def progress(msg):
        print(f"bench.py: {msg}", file=sys.stderr, flush=True)

    progress(f"{wl.name}: {value:.4g} grid-point z-steps/s, {wall / steps * 1e3:.4f} ms per step")
    extras = {}
    if not args.no_extras:
        wanted = None if args.extras == "all" else set(args.extras.split(","))
        for name, fn in (("adjoint", lambda: adjoint_ratio(dev)), ("batch", lambda: batch_ratio(dev)),
                         ("reduced_dims", lambda: reduced_dims(dev)),
                         ("diagnostics", lambda: diagnostics_cost(dev, wl)),
                         ("dk_map", lambda: dk_map_cost(dev)), ("paper_grids", lambda: paper_grids(dev))):
            if wanted is not None and name not in wanted:
                continue
            extras[name] = fn()
            progress(f"extra {name} done")

    cpu = None
    if not args.no_cpu_baseline:
        del fields, init
        torch.cuda.empty_cache()
        progress(f"oracle on {args.cpu_steps} steps of the CPU sample")
        cpu = cpu_baseline(wl, args.cpu_steps)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point·z-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded)",
        "config": {"workload": f"{wl.name}: {wl.nf}-field chi(2) split-step, "
                               f"{wl.nx}x{wl.ny}x{wl.nt} grid, {wl.nz} z-steps",
                   "nx": wl.nx, "ny": wl.ny, "nt": wl.nt, "nf": wl.nf, "nz": wl.nz,
                   "parallelism": "single GPU", "schedule": schedule},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "field_point_steps_per_s": value * wl.nf,
        "bytes_per_point_step": bytes_per_pt,
        "hbm_frac_step_wall": round(step_bytes / (wall / steps) / 1e9 / HBM_PEAK_GBS, 4),
        "event_ms_per_step": ev_ms / steps,
        "per_kernel": per_kernel,
        "fields_finite": finite,
        "adjoint_over_forward": extras.get("adjoint", {}).get("ratio"),
        "batched_over_sequential": extras.get("batch", {}).get("speedup"),
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
