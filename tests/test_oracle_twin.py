"""The two FP64 oracles, written separately from the paper (oracle/ssfm.py in
PyTorch, oracle/ssfm_numpy.py in NumPy), agree to rounding on small random
problems: two and three fields, constant dk and per-step profiles, loss and
third-order dispersion, a transverse mismatch map with and without a
per-step scale, odd and even axis lengths."""
import numpy as np
import pytest
import torch

from oracle import ssfm
from oracle.ssfm_numpy import NumpyOracle

KEYS = ("kappa", "diffraction", "tan_rho", "delay", "k2", "k3", "alpha")


def _case(seed, shape, nf, profile, tmap, scale):
    rng = np.random.default_rng(seed)
    nt, ny, nx = shape
    nz = 7
    params = [dict(kappa=rng.uniform(0.5, 2.0), diffraction=rng.uniform(0.1, 1.5),
                   tan_rho=rng.uniform(-0.6, 0.6), delay=rng.uniform(-1, 1), k2=rng.uniform(-2, 2),
                   k3=rng.uniform(-0.5, 0.5), alpha=rng.uniform(0, 0.3)) for _ in range(nf)]
    dz = 0.11
    dk_const = rng.uniform(-4, 4)
    dk = list(rng.uniform(-5, 5, nz)) if profile else None
    dk_map = rng.uniform(-3, 3, (ny, nx)) if tmap else None
    dk_scale = list(rng.uniform(-1, 2, nz)) if (tmap and scale) else None
    fields = [(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * 0.8 for _ in range(nf)]
    prob = ssfm.Problem(nx, ny, nt, nf, dz, [ssfm.FieldParams(**p) for p in params], dk_const=dk_const, dk=dk,
                        dk_map=dk_map, dk_map_scale=dk_scale)
    twin = NumpyOracle(nx, ny, nt, params, dz, dk_const=dk_const, dk=dk, dk_map=dk_map,
                       dk_map_scale=dk_scale)
    return prob, twin, fields, nz


@pytest.mark.parametrize("seed,shape,nf,profile,tmap,scale", [
    (1, (8, 6, 4), 2, False, False, False),
    (2, (5, 8, 8), 3, False, False, False),
    (3, (16, 16, 16), 2, True, False, False),
    (4, (4, 12, 9), 3, True, False, False),
    (5, (8, 8, 8), 2, False, True, False),
    (6, (6, 10, 16), 3, True, True, True),
    (7, (16, 4, 16), 2, True, True, True),
])
def test_numpy_twin_equals_torch_oracle(seed, shape, nf, profile, tmap, scale):
    prob, twin, fields, nz = _case(seed, shape, nf, profile, tmap, scale)
    a = ssfm.propagate([torch.from_numpy(f) for f in fields], prob, nz)
    b = twin.propagate(fields, nz)
    for x, y in zip(a, b):
        x = x.numpy()
        assert np.linalg.norm(x - y) <= 1e-12 * np.linalg.norm(y)
    # and the fields moved (the comparison is not of two identities)
    assert np.linalg.norm(b[0] - fields[0]) > 0.1 * np.linalg.norm(fields[0])
