"""The count sketch behind the whole-field parity checks (tests/sketch.py):
linear, chunking-independent, norm-preserving on average, and exact for an
error concentrated at a few points; the torch path equals the numpy one."""
import numpy as np
import torch

from tests.sketch import count_sketch, count_sketch_torch, sketched_rel_l2


def test_linear_and_chunk_independent():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(50_000) + 1j * rng.standard_normal(50_000)
    b = rng.standard_normal(50_000) + 1j * rng.standard_normal(50_000)
    sa, sb = count_sketch(a, 2048, 11), count_sketch(b, 2048, 11)
    assert np.allclose(count_sketch(a - 2 * b, 2048, 11), sa - 2 * sb, atol=1e-10)
    assert np.allclose(count_sketch(a, 2048, 11, chunk=777), sa, atol=1e-10)


def test_norm_estimate_spread_and_sparse():
    rng = np.random.default_rng(4)
    n, buckets = 1 << 20, 4096
    ratios = []
    for seed in range(8):
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        ratios.append(np.linalg.norm(count_sketch(x, buckets, seed)) / np.linalg.norm(x))
    ratios = np.array(ratios)
    # relative spread about 1/sqrt(2 B) = 1.1 %
    assert abs(ratios.mean() - 1) < 0.02 and ratios.std() < 0.03
    # an error at 20 points: all in distinct buckets (or nearly), norm kept
    x = np.zeros(n, dtype=np.complex128)
    x[rng.choice(n, 20, replace=False)] = rng.standard_normal(20) + 1j
    assert abs(np.linalg.norm(count_sketch(x, 16384, 5)) / np.linalg.norm(x) - 1) < 0.05


def test_relative_error_estimate_and_torch_path():
    rng = np.random.default_rng(5)
    r = rng.standard_normal((32, 64, 64)) + 1j * rng.standard_normal((32, 64, 64))
    e = 1e-5 * (rng.standard_normal(r.shape) + 1j * rng.standard_normal(r.shape))
    a = (r + e).astype(np.complex128)
    ref = count_sketch(r, 16384, 9)
    est = sketched_rel_l2(a, ref, float(np.sum(np.abs(r) ** 2)), 9)
    true = np.linalg.norm(e) / np.linalg.norm(r)
    assert abs(est / true - 1) < 0.05
    t = torch.from_numpy(a.astype(np.complex64))
    assert np.allclose(count_sketch_torch(t, 16384, 9), count_sketch(a.astype(np.complex64), 16384, 9),
                       rtol=0, atol=1e-9)
