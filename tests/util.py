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
    scale = None if wl.dk_map_scale is None else [float(v) for v in wl.dk_map_scale]
    return ssfm.Problem(wl.nx, wl.ny, wl.nt, wl.nf, wl.dz, fields,
                        dk_const=wl.dk_const, dk=dk, dk_map=wl.dk_map, dk_map_scale=scale)


def oracle_run(wl: inputs.Workload, nsteps=None, merge=False):
    """The oracle on a workload's entrance fields: the literal N/2 - L - N/2
    loop, or with adjacent half-steps merged (the reference of engine runs
    with merge_halves = 1)."""
    nsteps = wl.nz if nsteps is None else nsteps
    fn = ssfm.propagate_merged if merge else ssfm.propagate
    return fn([to_torch(a) for a in wl.init], oracle_problem(wl), nsteps)


def to_torch(a) -> torch.Tensor:
    return torch.from_numpy(np.asarray(a).astype(np.complex128))


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def bk_integral(sigma: float, xi: float) -> complex:
    """Boyd-Kleinman focusing integral int_{-xi}^{xi} exp(i sigma u)/(1 + i u) du
    by FP64 quadrature (real and imaginary parts separately)."""
    import math
    from scipy import integrate
    re = integrate.quad(lambda u: (math.cos(sigma * u) + u * math.sin(sigma * u)) / (1 + u * u), -xi, xi,
                        epsabs=1e-13, epsrel=1e-11, limit=400)[0]
    im = integrate.quad(lambda u: (math.sin(sigma * u) - u * math.cos(sigma * u)) / (1 + u * u), -xi, xi,
                        epsabs=1e-13, epsrel=1e-11, limit=400)[0]
    return complex(re, im)


def bk_efficiency(xi: float, dkl: float, diffraction: float, kappa_s: float = 1.0) -> float:
    """Closed-form undepleted CW SHG efficiency E_S / P_F^2 of a Gaussian beam
    focused at L/2 (grid cells of unit area): kappa_S^2 L |I|^2 / (8 pi D_F xi)
    with sigma = -dk z_R = -dk L / (2 xi)."""
    import math
    return kappa_s ** 2 * abs(bk_integral(-dkl / (2 * xi), xi)) ** 2 / (8 * math.pi * diffraction * xi)
