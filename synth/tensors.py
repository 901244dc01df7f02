"""Seeded random complex tensors for kernel-level tests and microbenchmarks."""
from __future__ import annotations

import numpy as np


def complex_normal(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Standard complex normal entries (E|z|^2 = 1) times ``scale``, complex128."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * (scale / np.sqrt(2.0))
