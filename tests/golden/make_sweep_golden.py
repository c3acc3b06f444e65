"""Write oracle reference data for all 64 instances of the seeded batched SHG
sweep (2 fields, grids 64^3 .. 128 x 128 x 256, 200-600 steps each).

Runs only the FP64 oracle (oracle/ssfm.py) on each instance's complex64
entrance fields and stores, per instance and field, the complex values at 512
seeded uniformly random points and at the 512 points of largest oracle
amplitude, the power trace P(tau), the energies, and a count sketch of the
whole field (tests/sketch.py; SKETCH_BUCKETS buckets, seed
SKETCH_SEED + 16 i + j) from which the GPU test estimates the whole-field
relative L2 error.

The instances take hours of CPU time in total, so the work can be split over
several processes: each call handles the instances i with i % parts == part
and keeps one file per instance in a scratch folder; a final call with
--merge collects them into shg_sweep_64.npz.

Usage: python -m tests.golden.make_sweep_golden <part> <parts> <scratch_dir> [threads]
       python -m tests.golden.make_sweep_golden --merge <scratch_dir>
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ssfm  # noqa: E402
from paper_2609_08384_amd import inputs  # noqa: E402
from tests.sketch import count_sketch  # noqa: E402
from tests.util import oracle_problem, to_torch  # noqa: E402

COUNT = 64
NSAMPLE = 512
SKETCH_BUCKETS = 4096
SKETCH_SEED = 9000
OUT = os.path.join(HERE, "shg_sweep_64.npz")


def _points(shape, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    return np.sort(rng.choice(n, size=min(NSAMPLE, n), replace=False))


def run_instance(i, wl):
    prob = oracle_problem(wl)
    out = ssfm.propagate([to_torch(a) for a in wl.init], prob, wl.nz)
    res = {"shape": np.array([wl.nx, wl.ny, wl.nt]), "nz": np.array(wl.nz),
           "uniform_idx": _points((wl.nt, wl.ny, wl.nx), 1000 + i),
           "energies": np.array(ssfm.energies(out, prob))}
    for j, a in enumerate(out):
        flat = a.reshape(-1)
        res[f"f{j}_uniform"] = flat[res["uniform_idx"]].numpy()
        top = torch.topk(flat.abs(), NSAMPLE).indices.sort().values
        res[f"f{j}_top_idx"] = top.numpy()
        res[f"f{j}_top"] = flat[top].numpy()
        res[f"f{j}_power"] = (a.abs() ** 2).sum(dim=(1, 2)).numpy()
        res[f"f{j}_sketch"] = count_sketch(a, SKETCH_BUCKETS, SKETCH_SEED + 16 * i + j).astype(np.complex64)
    return res


def main():
    if sys.argv[1] == "--merge":
        scratch = sys.argv[2]
        merged = {}
        for i in range(COUNT):
            with np.load(os.path.join(scratch, f"inst{i:02d}.npz")) as d:
                for k in d.files:
                    merged[f"i{i:02d}_{k}"] = d[k]
        np.savez_compressed(OUT, **merged)
        print("wrote", OUT, flush=True)
        return
    part, parts, scratch = int(sys.argv[1]), int(sys.argv[2]), sys.argv[3]
    if len(sys.argv) > 4:
        torch.set_num_threads(int(sys.argv[4]))
    os.makedirs(scratch, exist_ok=True)
    wls = inputs.shg_sweep()
    for i, wl in enumerate(wls):
        path = os.path.join(scratch, f"inst{i:02d}.npz")
        if i % parts != part or os.path.exists(path):
            continue
        t0 = time.time()
        res = run_instance(i, wl)
        np.savez_compressed(path + ".tmp.npz", **res)
        os.replace(path + ".tmp.npz", path)
        print(f"instance {i}: {wl.nx}x{wl.ny}x{wl.nt}, {wl.nz} steps, {time.time() - t0:.0f} s",
              flush=True)


if __name__ == "__main__":
    main()
