"""Write oracle reference gradients for the inverse-design workload
(SHG 128 x 128 x 64, 400 steps, per-step dk profile): J = -sum |S(L)|^2 and
its gradients with respect to the input fields and the dk profile, from the
oracle's own adjoint (oracle/adjoint.py, reverse-mode through the FP64 loop).
Stores J, the full dJ/ddk, dJ/dF_in at 4096 uniform and 4096 largest points,
the transverse-summed |dJ/dF_in|^2 per tau, its squared norm and a count
sketch of the whole gradient (tests/sketch.py; SKETCH_BUCKETS buckets, seed
SKETCH_SEED).
Usage: python -m tests.golden.make_adjoint_golden [threads]
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import adjoint as oadj  # noqa: E402
from paper_2609_08384_amd import inputs  # noqa: E402
from tests.golden.make_golden import sample_points  # noqa: E402
from tests.sketch import count_sketch  # noqa: E402
from tests.util import oracle_problem  # noqa: E402

SKETCH_BUCKETS = 16384
SKETCH_SEED = 8000


def main():
    if len(sys.argv) > 1:
        torch.set_num_threads(int(sys.argv[1]))
    wl = inputs.shg_adjoint()
    prob = oracle_problem(wl)
    t0 = time.time()
    j, g, gdk = oadj.gradients([torch.from_numpy(a) for a in wl.init], list(wl.dk), prob, wl.nz,
                               loss=lambda out, p: -(out[1].abs() ** 2).sum())
    print(f"J = {j}  ({time.time() - t0:.0f} s)", flush=True)
    gf = g[0].reshape(-1)
    uni = sample_points(g[0].shape)
    top = torch.topk(gf.abs(), 4096).indices.sort().values
    np.savez_compressed(os.path.join(HERE, "shg_adjoint_grad.npz"), J=np.array(j), grad_dk=gdk.numpy(),
                        uniform_idx=uni, gF_uniform=gf[uni].numpy(), top_idx=top.numpy(),
                        gF_top=gf[top].numpy(), gF_power=(g[0].abs() ** 2).sum(dim=(1, 2)).numpy(),
                        gF_norm2=np.array(float((g[0].abs() ** 2).sum())),
                        gF_sketch=count_sketch(g[0], SKETCH_BUCKETS, SKETCH_SEED).astype(np.complex64))
    print("wrote shg_adjoint_grad.npz", flush=True)


if __name__ == "__main__":
    main()
