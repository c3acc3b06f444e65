"""Schedule autotuner: picks, per grid shape and field count, the plan
schedule (see brahms_schedule in include/brahms.h) that runs fastest on this
GPU, by timing each candidate on scratch fields, and caches the choice.

This is the plan-by-measurement idea of the paper's CPU backend (FFTW
planning with measurement, Sec. 5.1) applied to the GPU schedules.  The
timing loop only calls the C ABI; every candidate computes the same result to
rounding.

Merged RK4 half-steps (schedule field merge_halves) are not a trade-off to
measure: they take one RK4 update per step instead of two and change the
result by O(dz^5) per step, far below FP32 rounding.  The tuner turns them on
wherever the plan allows them (a constant dk and no transverse map) unless
asked not to, and times the other fields with them.  Fused step pairs (two
passes per step instead of three, same arithmetic) are a trade of HBM
traffic for register pressure and are timed like the pass orders.
"""
from __future__ import annotations

import json
import os
import threading
import time
from typing import Dict, Optional

import torch

from . import brahms

CANDIDATES = [{"pass_order": o, "graph": g} for g in (0, 1) for o in (0, 1, 2, 3)]
ROUNDS = 3   # timing rounds per candidate (the best is kept)
_lock = threading.Lock()
_memo: Dict[str, dict] = {}


def cache_path() -> str:
    root = os.environ.get("BRAHMS_CACHE_DIR") or os.path.join(
        os.path.expanduser("~"), ".cache", "brahms")
    return os.path.join(root, "schedules.json")


def _arch(device) -> str:
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def _key(arch: str, nx: int, ny: int, nt: int, nf: int, merge: int) -> str:
    return f"v8:{arch}:{nx}x{ny}x{nt}:nf{nf}:m{merge}"


def split_masks(nx: int, ny: int, nt: int):
    """Every choice of register/lane split (schedule field split) that
    changes something for this shape: subsets of the axes whose length has a
    second split (long tau axes keep theirs)."""
    bits = [1 << a for a, n in enumerate((nx, ny, nt)) if n in brahms.ALT_SPLIT_LENGTHS]
    masks = [0]
    for b in bits:
        masks += [m | b for m in masks]
    return masks


def wide_masks(schedule: dict, nx: int, ny: int, nt: int):
    """Values of the schedule field `wide` worth timing: each axis whose
    passes are linear in this schedule (the middle axis; with merged
    half-steps and no fused pairs also the first), alone and together;
    none for long tau axes, and none on axes of length 1 or of a length
    without a wide form (brahms.NARROW_ONLY_LENGTHS)."""
    if nt > 256:
        return []
    order = [(0, 1, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)][schedule["pass_order"]]
    linear = [order[1]]
    if schedule.get("merge_halves") and not schedule.get("fuse_steps"):
        linear.append(order[0])
    shape = (nx, ny, nt)
    bits = [1 << a for a in linear if shape[a] > 1 and shape[a] not in brahms.NARROW_ONLY_LENGTHS]
    masks = list(bits)
    if len(bits) > 1:
        masks.append(sum(bits))
    return masks


def can_merge(params: brahms.Params) -> bool:
    """Whether a plan with these parameters accepts merge_halves = 1."""
    return params.dk is None and getattr(params, "dk_map", None) is None


def can_fuse(nx: int, ny: int, nt: int) -> bool:
    """Whether a plan of this shape has x and y passes at the ends of a step
    (and so accepts fuse_steps = 1 with merged half-steps): every shape but
    plane waves with a single tau pass."""
    return nt > 256 or not (nx == 1 and ny == 1)


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(entries: dict):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(entries, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def measure(nx: int, ny: int, nt: int, nf: int, params: brahms.Params, schedule: dict,
            device="cuda:0", steps: int = 64, warmup: int = 8) -> float:
    """Milliseconds per z-step of one schedule on scratch fields (one whole
    64-step chunk, the unit a graph schedule replays)."""
    gen = torch.Generator(device="cpu").manual_seed(1234)
    fields = [(0.1 * torch.randn(nt, ny, nx, dtype=torch.complex64, generator=gen)).to(device)
              for _ in range(nf)]
    plan = brahms.Plan(nx, ny, nt, nf, params)
    plan.set_schedule(**schedule)
    plan.bind(fields)
    plan.step(warmup)
    torch.cuda.synchronize(device)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    plan.step(steps)
    ev1.record()
    torch.cuda.synchronize(device)
    plan.destroy()
    return ev0.elapsed_time(ev1) / steps


def tune(nx: int, ny: int, nt: int, nf: int, params: brahms.Params, device="cuda:0",
         refresh: bool = False, merge_halves: bool = True) -> dict:
    """Best schedule for this shape (cached in memory and on disk)."""
    arch = _arch(device)
    merge = int(merge_halves and can_merge(params))
    key = _key(arch, nx, ny, nt, nf, merge)
    with _lock:
        if not refresh:
            if key in _memo:
                return _memo[key]
            disk = _load()
            if key in disk:
                _memo[key] = disk[key]["schedule"]
                return _memo[key]
        # time with the same linear coefficients but no coupling blow-up risk
        scratch = brahms.Params(dz=params.dz, fields=params.fields, dk_const=params.dk_const,
                                dk=None, dx=params.dx, dy=params.dy, dt=params.dt)
        fuses = (0, 1) if merge and can_fuse(nx, ny, nt) else (0,)
        cands = [dict(c, merge_halves=merge, fuse_steps=f) for f in fuses for c in CANDIDATES]
        # the candidates differ by a few per cent: a warm-up run brings the
        # clocks up first, and each candidate keeps the best of ROUNDS
        # interleaved rounds (a slow round on a throttled clock then hits
        # every candidate alike)
        measure(nx, ny, nt, nf, scratch, cands[-1], device, steps=4 * 64)
        best_of = [float("inf")] * len(cands)
        for _ in range(ROUNDS):
            for i, c in enumerate(cands):
                best_of[i] = min(best_of[i], measure(nx, ny, nt, nf, scratch, c, device))
        times = list(zip(best_of, cands))
        best_ms, best = min(((t, c) for t, c in times if not c["graph"]), key=lambda tc: tc[0])
        # a graph pays off only where launches are a visible cost: take it
        # when it is at least 2 % faster than the best launch-by-launch order
        g_ms, g = min(((t, c) for t, c in times if c["graph"]), key=lambda tc: tc[0])
        if g_ms < 0.98 * best_ms:
            best_ms, best = g_ms, g
        # the register/lane splits of the axes that have two, on the best
        # schedule so far (it picks lines per block against values per lane)
        for mask in split_masks(nx, ny, nt)[1:]:
            c = dict(best, split=mask)
            t = min(measure(nx, ny, nt, nf, scratch, c, device) for _ in range(ROUNDS))
            times.append((t, c))
            if t < best_ms:
                best_ms, best = t, c
        # 512-thread blocks for the linear passes, on the axes whose passes
        # are linear in the best schedule
        for mask in wide_masks(best, nx, ny, nt):
            c = dict(best, wide=mask)
            t = min(measure(nx, ny, nt, nf, scratch, c, device) for _ in range(ROUNDS))
            times.append((t, c))
            if t < best_ms:
                best_ms, best = t, c
        _memo[key] = dict(best)
        disk = _load()
        disk[key] = {"schedule": dict(best), "ms_per_step": best_ms,
                     "candidates": [{"schedule": c, "ms_per_step": t} for t, c in times]}
        _store(disk)
        return _memo[key]


def apply(plan: brahms.Plan, device="cuda:0", merge_halves: bool = True) -> dict:
    """Tune (or look up) the plan's shape and set the chosen schedule."""
    sched = tune(plan.nx, plan.ny, plan.nt, plan.nf, plan.params, device, merge_halves=merge_halves)
    plan.set_schedule(**sched)
    return sched


GROUP_CANDIDATES = (0, 1 << 30)   # cache-budget groups, or every same-shape problem at once
LIMIT_CANDIDATES = (0, 1, 2, 4, 1 << 30)   # per-shape launch-group sizes
# one captured graph, or launches issued on 2 or 4 streams (all groups at
# once, or the largest group after the others)
STREAM_CANDIDATES = ((1, 0), (2, 0), (4, 0), (3, 1), (4, 1))


def _probe_time(batch: "brahms.Batch", fields, device) -> float:
    """Milliseconds of one run of an already scheduled batch (after a
    warm-up run that also builds its graph)."""
    batch.bind(fields)
    batch.run()
    torch.cuda.synchronize(device)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    batch.run()
    ev1.record()
    torch.cuda.synchronize(device)
    return ev0.elapsed_time(ev1)


def tune_batch(batch: "brahms.Batch", device="cuda:0", max_steps: int = 64,
               merge_halves: bool = True, run_fields=None, refine: int = 6) -> dict:
    """Pick the pass orders, the launch-group sizes and the launch mode of a
    batch by timing copies of it on scratch fields, with at most max_steps
    steps per problem:
    * per grid shape, the register/lane splits and the 512-thread linear x
      and y passes that `tune` found fastest for a plain solve;
    * per grid shape alone, the group sizes LIMIT_CANDIDATES (the fastest
      differs between shapes: small grids want many problems per launch,
      large ones few);
    * the whole batch with those per-shape sizes, and with the global sizes
      GROUP_CANDIDATES, each with the per-shape orders of `tune` (the fastest
      for a plain solve) and with one order for every problem, each as one
      captured graph (groups in sequence) and with its launches issued on
      STREAM_CANDIDATES streams (groups of different shapes at the same
      time, where concurrent groups compete for the chip, so the best order
      or group size alone need not be the best together).
    Merged half-steps are taken when every problem allows them; fused step
    pairs are timed against three passes per step on the fastest choice.
    With `run_fields` (the caller's fields of the batch, per problem a list
    of tensors) the `refine` fastest candidates are then timed on `batch`
    itself, each over a whole run on those fields (saved first and restored
    before every run) by wall clock, and the fastest of those is taken: the
    short probes rank the launch modes, but a whole ragged run can order the
    first few otherwise (and events on the caller's stream read runs on
    several streams short).
    Applies the chosen schedule to `batch`."""
    problems = batch.problems
    n = len(problems)
    merge = int(merge_halves and all(can_merge(prm) for (_, _, _, _, prm, _) in problems))
    # (batches holding a long tau problem do not fuse)
    fuse = int(merge and all(nt <= 256 for (_, _, nt, _, _, _) in problems) and
               any(can_fuse(nx, ny, nt) for (nx, ny, nt, _, _, _) in problems))
    fuse_ok = fuse
    sched = [tune(nx, ny, nt, nf, prm, device, merge_halves=bool(merge))
             for (nx, ny, nt, nf, prm, _) in problems]
    tuned = [sc["pass_order"] for sc in sched]
    splits = [sc.get("split", 0) for sc in sched]
    # (a batch's linear tau passes keep 256-thread blocks)
    wides = [sc.get("wide", 0) & 3 for sc in sched]
    order_sets = {"per_shape": tuned, "all_0": [0] * n, "all_1": [1] * n}
    short = [(nx, ny, nt, nf, prm, min(ns, max_steps)) for (nx, ny, nt, nf, prm, ns) in problems]
    gen = torch.Generator(device="cpu").manual_seed(7)
    fields = [[(0.1 * torch.randn(nt, ny, nx, dtype=torch.complex64, generator=gen)).to(device)
               for _ in range(nf)] for (nx, ny, nt, nf, _, _) in problems]
    # per-shape group sizes
    shapes = {}
    for i, (nx, ny, nt, nf, _, _) in enumerate(problems):
        shapes.setdefault((nx, ny, nt, nf), []).append(i)
    limits = [0] * n
    shape_ms = {}
    for key, idx in shapes.items():
        sub = brahms.Batch([short[i] for i in idx])
        sub.set_merge_halves(merge)
        sub.set_fuse_steps(fuse)
        sub.set_splits([splits[i] for i in idx])
        sub.set_wide([wides[i] for i in idx])
        sub.set_schedule(0, [tuned[i] for i in idx])
        times = []
        for lim in LIMIT_CANDIDATES:
            sub.set_group_limits([lim] * len(idx))
            times.append((_probe_time(sub, [fields[i] for i in idx], device), lim))
        sub.destroy()
        best_ms, best_lim = min(times)
        for i in idx:
            limits[i] = best_lim
        shape_ms["%dx%dx%d:nf%d" % key] = {str(l): t for t, l in times}
    # the whole batch
    probe = brahms.Batch(short)
    probe.set_merge_halves(merge)
    probe.set_fuse_steps(fuse)
    probe.set_splits(splits)
    probe.set_wide(wides)
    candidates = []

    def configure(gm, oname):
        if gm is None:
            probe.set_schedule(0, order_sets[oname])
            probe.set_group_limits(limits)
        else:
            probe.set_group_limits(None)
            probe.set_schedule(gm, order_sets[oname])

    for streams in STREAM_CANDIDATES:
        probe.set_streams(*streams)
        configure(None, "per_shape")
        candidates.append((_probe_time(probe, fields, device), "per_shape_limits", None, "per_shape", streams))
        for gm in GROUP_CANDIDATES:
            for name in order_sets:
                configure(gm, name)
                candidates.append((_probe_time(probe, fields, device), f"group_max={gm}", gm, name, streams))
    best = min(candidates, key=lambda c: c[0])
    _, label, gm, oname, streams = best
    if fuse:
        # the same choice with three passes per step
        probe.set_fuse_steps(0)
        probe.set_streams(*streams)
        configure(gm, oname)
        t3 = _probe_time(probe, fields, device)
        candidates.append((t3, label + "/three_passes", gm, oname, streams))
        if t3 < best[0]:
            fuse = 0
    probe.destroy()

    def apply(c_fuse, c_streams, c_gm, c_oname):
        batch.set_merge_halves(merge)
        batch.set_fuse_steps(c_fuse)
        batch.set_splits(splits)
        batch.set_wide(wides)
        batch.set_streams(*c_streams)
        if c_gm is None:
            batch.set_schedule(0, order_sets[c_oname])
            batch.set_group_limits(limits)
        else:
            batch.set_group_limits(None)
            batch.set_schedule(c_gm, order_sets[c_oname])

    whole_ms = {}
    if run_fields is not None and refine > 0:
        saved = [[f.clone() for f in fs] for fs in run_fields]

        def restore():
            for fs, ss in zip(run_fields, saved):
                for f, g in zip(fs, ss):
                    f.copy_(g)
            torch.cuda.synchronize(device)

        timed = []
        for c in sorted(candidates, key=lambda c: c[0])[:refine]:
            c_fuse = 0 if c[1].endswith("/three_passes") else fuse_ok
            apply(c_fuse, c[4], c[2], c[3])
            batch.bind(run_fields)
            batch.run()                      # builds the graphs
            torch.cuda.synchronize(device)
            restore()
            t0 = time.perf_counter()
            batch.run()
            torch.cuda.synchronize(device)
            t = (time.perf_counter() - t0) * 1e3
            timed.append((t, c, c_fuse))
            whole_ms[f"{c[1]}/{c[3]}/streams={c[4][0]}{'/largest_alone' if c[4][1] else ''}"] = t
        restore()
        _, (_, label, gm, oname, streams), fuse = min(timed, key=lambda x: x[0])
    apply(fuse, streams, gm, oname)
    return {"choice": label, "group_max": gm, "group_limits": limits if gm is None else None,
            "pass_orders": order_sets[oname], "orders": oname, "merge_halves": merge, "fuse_steps": fuse,
            "splits": splits,
            "wide": wides,
            "streams": streams,
            "probe_ms": {f"{c[1]}/{c[3]}/streams={c[4][0]}{'/largest_alone' if c[4][1] else ''}": c[0]
                         for c in candidates},
            "shape_probe_ms": shape_ms,
            "whole_run_ms": whole_ms}
