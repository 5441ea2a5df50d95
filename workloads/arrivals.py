"""Seeded Poisson arrival trace for the served stream.

Request r arrives after exponential inter-arrival gaps of mean ``1/rate``;
its qubit count is uniform over ``sizes``; it uses Hamiltonian seed
``h_seed_base + r`` and amplitude seed ``t_seed_base + r``.
"""
from __future__ import annotations

import numpy as np


def poisson_requests(count: int, rate_per_s: float, seed: int,
                     sizes=(12, 16, 20, 24, 26),
                     h_seed_base: int = 1_000_000, t_seed_base: int = 2_000_000):
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrival = np.cumsum(gaps)
    ns = rng.choice(np.asarray(sizes), size=count)
    return [
        {"id": r, "t_arrival": float(arrival[r]), "n_qubits": int(ns[r]),
         "n_electrons": int(ns[r]) // 2, "h_seed": h_seed_base + r, "theta_seed": t_seed_base + r}
        for r in range(count)
    ]
