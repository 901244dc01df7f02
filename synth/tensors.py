"""Seeded random complex tensors for kernel-level tests and microbenchmarks."""
from __future__ import annotations

import numpy as np


def complex_normal(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Standard complex normal entries (E|z|^2 = 1) times ``scale``, complex128."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * (scale / np.sqrt(2.0))


def complex_normal_c64(n: int, seed: int, chunk: int = 1 << 24) -> np.ndarray:
    """n standard complex normal entries as complex64, drawn in chunks (for
    tensors too large to build in complex128 first); one seeded stream."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.complex64)
    f = out.view(np.float32)
    for s in range(0, 2 * n, 2 * chunk):
        e = min(2 * n, s + 2 * chunk)
        f[s:e] = rng.standard_normal(e - s, dtype=np.float32) * np.float32(1.0 / np.sqrt(2.0))
    return out
