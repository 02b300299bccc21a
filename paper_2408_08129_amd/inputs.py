"""Seeded synthetic inputs shared by the GPU path and the oracle (no method arithmetic here)."""
from __future__ import annotations

import numpy as np


def random_state(nf: int, n: int, seed: int, wind: float = 10.0) -> np.ndarray:
    """Conserved variables (rho, m..., rho E) per node with rho in [0.8, 1.2], momentum components
    up to +-wind*rho and a total energy around 2.5e5 J/m^3, so that pressure stays positive."""
    rng = np.random.default_rng(seed)
    U = np.zeros((nf, n))
    U[0] = 1.0 + 0.2 * rng.uniform(-1.0, 1.0, n)
    for l in range(1, nf - 1):
        U[l] = U[0] * wind * rng.uniform(-1.0, 1.0, n)
    U[nf - 1] = 2.5e5 * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, n))
    return U


def random_positive(n: int, seed: int, lo: float, hi: float) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


def random_normal(n: int, seed: int, sigma: float = 1.0) -> np.ndarray:
    return sigma * np.random.default_rng(seed).standard_normal(n)
