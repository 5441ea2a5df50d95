"""Random Pauli rotations and Pauli sums for the raw-sweep workload.

Strings are returned as packed ``uint64`` masks ``(x, z)``: bit q of ``x`` is
set when the factor on qubit q is X or Y, bit q of ``z`` when it is Z or Y.

* ``random_rotations``: each rotation acts on exactly 4 distinct qubits drawn
  uniformly, with factors X/Y only and an odd number of Y (the 8 such
  patterns, uniform), like a JW double-excitation string without its Z tail;
  angles ``phi ~ U[-a, a]``.
* ``random_pauli_sum``: weight ``w ~ U{1..4}``, distinct uniform qubits, each
  factor uniform in {X, Y, Z}, coefficient ``c ~ U[-1, 1]``.  A string that
  was already drawn is rejected and drawn again, so the strings are distinct.
"""
from __future__ import annotations

from math import comb

import numpy as np

# the 8 X/Y patterns on 4 qubits with an odd number of Y (1 = Y, 0 = X)
_ODD_Y = [p for p in range(16) if bin(p).count("1") % 2 == 1]


def random_rotations(n_qubits: int, count: int, seed: int, amplitude: float = 0.1):
    rng = np.random.default_rng(seed)
    x = np.zeros(count, dtype=np.uint64)
    z = np.zeros(count, dtype=np.uint64)
    for k in range(count):
        qs = rng.choice(n_qubits, size=4, replace=False)
        pat = _ODD_Y[int(rng.integers(8))]
        xm = 0
        zm = 0
        for t, q in enumerate(qs):
            xm |= 1 << int(q)
            if (pat >> t) & 1:
                zm |= 1 << int(q)
        x[k] = xm
        z[k] = zm
    phi = rng.uniform(-amplitude, amplitude, size=count)
    return x, z, phi


def random_pauli_sum(n_qubits: int, count: int, seed: int):
    available = sum(comb(n_qubits, w) * 3 ** w for w in range(1, min(4, n_qubits) + 1))
    if count > available:
        raise ValueError(f"only {available} distinct strings of weight <= 4 on {n_qubits} qubits")
    rng = np.random.default_rng(seed)
    seen = set()
    xs, zs, cs = [], [], []
    while len(xs) < count:
        w = int(rng.integers(1, 5))
        qs = rng.choice(n_qubits, size=w, replace=False)
        kinds = rng.integers(0, 3, size=w)  # 0 = X, 1 = Y, 2 = Z
        xm = 0
        zm = 0
        for q, kd in zip(qs, kinds):
            if kd in (0, 1):
                xm |= 1 << int(q)
            if kd in (1, 2):
                zm |= 1 << int(q)
        c = rng.uniform(-1.0, 1.0)
        if (xm, zm) in seen:
            continue
        seen.add((xm, zm))
        xs.append(xm)
        zs.append(zm)
        cs.append(c)
    return np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64), np.array(cs)
