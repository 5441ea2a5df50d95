"""Seeded UCCSD amplitudes: ``theta ~ U[-a, a]`` drawn as one vector."""
from __future__ import annotations

import numpy as np


def uniform_amplitudes(n_params: int, amplitude: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=int(n_params)).astype(np.float64)
