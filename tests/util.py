"""Glue between the seeded workloads and the oracle (tests only)."""
import numpy as np
import torch

from oracle import ssfm
from paper_2609_08384_amd import inputs


def oracle_problem(wl: inputs.Workload) -> ssfm.Problem:
    fields = [ssfm.FieldParams(kappa=f.kappa, diffraction=f.diffraction,
                               tan_rho=f.tan_rho, delay=f.delay, k2=f.k2,
                               k3=f.k3, alpha=f.alpha) for f in wl.fields]
    dk = None if wl.dk is None else [float(v) for v in wl.dk]
    return ssfm.Problem(wl.nx, wl.ny, wl.nt, wl.nf, wl.dz, fields,
                        dk_const=wl.dk_const, dk=dk)


def to_torch(a) -> torch.Tensor:
    return torch.from_numpy(np.asarray(a).astype(np.complex128))


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))
