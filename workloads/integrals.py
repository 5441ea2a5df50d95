"""Seeded synthetic molecular integrals (stand-in for the PySCF integrals of
Section 3.1; no molecular data is reproduced).

Recipe, with the draw order part of the definition:

* ``M = n_qubits // 2`` spatial orbitals.
* ``h[p, p] = -1 + 0.5 * p / M + 0.05 * u``  for p = 0..M-1 in order.
* ``h[p, q] = h[q, p] = 0.1 * u * exp(-|p - q|)`` for p = 1..M-1, q = 0..p-1.
* Two-electron integrals in chemist's notation ``(pq|rs)`` with the 8-fold
  permutational symmetry.  Canonical quadruples ``p >= q``, ``r >= s``,
  ``pq >= rs`` (``pq = p(p+1)/2 + q``) are visited in lexicographic order of
  ``(p, q, r, s)``; each draws one ``u`` and sets

    - ``(pp|rr) = 0.5 * exp(-|p - r|) * (1 + 0.1 * u)``  (Coulomb-like), else
    - ``(pq|rs) = 0.1 * u * exp(-|p - r|)``,

  then copies the value to all 8 images.  The decay is evaluated on the
  canonical representative because ``|p - r|`` is not symmetry invariant.

Here ``u ~ U(-1, 1)`` from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math

import numpy as np


def synthetic_integrals(n_qubits: int, seed: int):
    """Return ``(h, eri)``: ``h`` is (M, M), ``eri`` is (M, M, M, M) chemist's
    notation, both float64, for ``M = n_qubits // 2`` spatial orbitals."""
    if n_qubits < 2 or n_qubits % 2:
        raise ValueError("n_qubits must be even and >= 2")
    M = n_qubits // 2
    rng = np.random.default_rng(seed)
    h = np.zeros((M, M))
    for p in range(M):
        h[p, p] = -1.0 + 0.5 * p / M + 0.05 * rng.uniform(-1.0, 1.0)
    for p in range(1, M):
        for q in range(p):
            v = 0.1 * rng.uniform(-1.0, 1.0) * math.exp(-abs(p - q))
            h[p, q] = v
            h[q, p] = v
    eri = np.zeros((M, M, M, M))
    for p in range(M):
        for q in range(p + 1):
            pq = p * (p + 1) // 2 + q
            for r in range(M):
                for s in range(r + 1):
                    rs = r * (r + 1) // 2 + s
                    if pq < rs:
                        continue
                    u = rng.uniform(-1.0, 1.0)
                    if p == q and r == s:
                        v = 0.5 * math.exp(-abs(p - r)) * (1.0 + 0.1 * u)
                    else:
                        v = 0.1 * u * math.exp(-abs(p - r))
                    for a, b, c, d in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                                       (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
                        eri[a, b, c, d] = v
    return h, eri
