"""Signed-hash sketches of whole fields (tests only).

A count sketch maps a field a (any shape, read in its flat index order) to
B buckets: S(a)[b] = sum over grid points i with h(i) = b of s(i) a_i, with
the bucket h(i) and the sign s(i) = +-1 taken from a seeded 64-bit hash of
the index.  It is linear, S(a) - S(r) = S(a - r), and E ||S(x)||^2 = ||x||^2
for any x; an x whose mass sits at a few points (the error of a tightly
focused beam) lands in distinct buckets and keeps its norm almost exactly,
and a spread-out x is estimated with a relative standard deviation of about
1/sqrt(2 B).  So ||S(a) - S(r)|| / ||r|| estimates the whole-field relative
L2 error from B stored numbers instead of every grid value.

The reference sketches are written by the scripts in tests/golden from the
oracle's fields; the GPU tests sketch their own output the same way.
"""
from __future__ import annotations

import numpy as np

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_GOLD = np.uint64(0x9E3779B97F4A7C15)


def _mix(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (wrapping uint64 arithmetic)."""
    x = x ^ (x >> np.uint64(30))
    x = x * _M1
    x = x ^ (x >> np.uint64(27))
    x = x * _M2
    return x ^ (x >> np.uint64(31))


def bucket_signs(n: int, buckets: int, seed: int, start: int = 0):
    """Bucket index and sign of grid points start .. start + n - 1."""
    idx = np.arange(start, start + n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        h = _mix(idx * _GOLD + np.uint64(seed) * _M2 + np.uint64(1))
    b = (h % np.uint64(buckets)).astype(np.int64)
    s = np.where((h >> np.uint64(63)) == 0, 1.0, -1.0)
    return b, s


_NP_CACHE = {}


def _cached(n: int, buckets: int, seed: int):
    key = (n, buckets, seed)
    if key not in _NP_CACHE:
        if len(_NP_CACHE) >= 6:   # a few fields' hashes at a time
            _NP_CACHE.pop(next(iter(_NP_CACHE)))
        _NP_CACHE[key] = bucket_signs(n, buckets, seed)
    return _NP_CACHE[key]


def count_sketch(a, buckets: int, seed: int, chunk: int = 0) -> np.ndarray:
    """The complex128 sketch of a complex array (numpy or torch, any shape);
    chunk > 0 hashes the indices in pieces of that size instead of caching
    the hash of the whole index range."""
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    flat = np.asarray(a).reshape(-1)
    out = np.zeros(buckets, dtype=np.complex128)
    step = chunk if chunk > 0 else max(1, flat.size)
    for lo in range(0, flat.size, step):
        part = flat[lo:lo + step]
        b, s = bucket_signs(part.size, buckets, seed, lo) if chunk > 0 else _cached(part.size, buckets, seed)
        out.real += np.bincount(b, weights=s * part.real.astype(np.float64), minlength=buckets)
        out.imag += np.bincount(b, weights=s * part.imag.astype(np.float64), minlength=buckets)
    return out


def sketched_rel_l2(a, ref_sketch: np.ndarray, ref_norm2: float, seed: int) -> float:
    """Estimated ||a - r|| / ||r|| from r's stored sketch and its exact squared norm."""
    sa = count_sketch(a, ref_sketch.size, seed)
    return float(np.linalg.norm(sa - ref_sketch) / np.sqrt(ref_norm2))


_CACHE = {}


def count_sketch_torch(t, buckets: int, seed: int):
    """The same sketch of a complex torch tensor, summed on its own device in
    float64 (equal to count_sketch up to the order of the additions)."""
    import torch

    key = (t.numel(), buckets, seed, str(t.device))
    if key not in _CACHE:
        b, s = bucket_signs(t.numel(), buckets, seed)
        if len(_CACHE) >= 6:   # a few fields' hashes at a time
            _CACHE.pop(next(iter(_CACHE)))
        _CACHE[key] = (torch.from_numpy(b).to(t.device), torch.from_numpy(s).to(t.device))
    b, s = _CACHE[key]
    flat = t.reshape(-1)
    re = torch.zeros(buckets, dtype=torch.float64, device=t.device)
    im = torch.zeros(buckets, dtype=torch.float64, device=t.device)
    re.index_add_(0, b, s * flat.real.double())
    im.index_add_(0, b, s * flat.imag.double())
    return (re.cpu().numpy() + 1j * im.cpu().numpy())
