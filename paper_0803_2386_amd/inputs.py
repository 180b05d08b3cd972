"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no transform arithmetic: it only draws numbers.  The tests
and the benchmark feed the same arrays to the HIP path and to the CPU oracle.

The paper times transforms of synthetic vectors of length 2^2 .. 2^24 and
never states their distribution (its worked examples use iota n); the
stand-in here is real and imaginary parts i.i.d. uniform on [-1, 1), drawn in
float64 from numpy's default_rng(seed) and rounded once to the working
precision.  Uneven batches draw their log2-lengths uniformly.
"""
from __future__ import annotations

import numpy as np

WORKLOADS = {
    "c128_n1024": dict(n=1 << 10, batch=1, dtype="complex128", lift=None),
    "c64_n2^24_lift4096x4096": dict(n=1 << 24, batch=1, dtype="complex64", lift=(4096, 4096)),
    "c64_uneven8192_2^6..2^14": dict(count=8192, kmin=6, kmax=14, dtype="complex64"),
    "c64_b256_n2^16_lift256x256": dict(n=1 << 16, batch=256, dtype="complex64", lift=(256, 256)),
    "c64_b256_n2^20_radix16": dict(n=1 << 20, batch=256, dtype="complex64", lift=(256, 4096)),
}


def uniform_complex(shape, seed: int = 0, dtype=np.complex64) -> np.ndarray:
    """Re/im i.i.d. U[-1, 1) drawn in float64 from default_rng(seed), then cast."""
    rng = np.random.default_rng(seed)
    shape = (shape,) if np.isscalar(shape) else tuple(shape)
    re = rng.uniform(-1.0, 1.0, shape)
    im = rng.uniform(-1.0, 1.0, shape)
    out = np.empty(shape, dtype=np.complex128)
    out.real = re
    out.imag = im
    return out.astype(dtype)


def uneven_sizes(count: int = 8192, kmin: int = 6, kmax: int = 14, seed: int = 0) -> np.ndarray:
    """Lengths 2^k with k uniform on {kmin..kmax}, in draw order."""
    rng = np.random.default_rng(seed + 7919)
    return (1 << rng.integers(kmin, kmax + 1, count)).astype(np.int64)


def loss_weights(n: int, seed: int = 0) -> np.ndarray:
    """w_k i.i.d. U[0, 1) for the weighted-power loss."""
    return np.random.default_rng(seed + 104729).uniform(0.0, 1.0, n)


def device_uniform_complex(numel: int, seed: int, dtype, device):
    """Large inputs drawn directly on the device: re/im U[-1, 1) from torch's
    seeded generator (used where a host draw would not fit the time budget;
    the oracle then reads the same values back)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    real = torch.float32 if dtype == torch.complex64 else torch.float64
    x = torch.empty(2 * int(numel), dtype=real, device=device)
    x.uniform_(-1.0, 1.0, generator=g)
    return x.view(dtype)
