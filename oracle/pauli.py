"""Pauli strings packed as two bit masks (oracle).

A string on n qubits is ``(x, z)``: bit q of ``x`` is set when the factor on
qubit q is X or Y, bit q of ``z`` when it is Z or Y.  The operator is
``P = i^{|x & z|} X^x Z^z`` (|.| = popcount), which is the tensor product of
the single-qubit factors with no extra phase.  Qubit q is bit q of a basis
index k (little-endian), so ``X^x Z^z |k> = (-1)^{|k & z|} |k ^ x>``.

The paper's Hamiltonian (Eq. 1, Section 3.1) is a real combination of such
strings.
"""
from __future__ import annotations

import numpy as np

_I2 = np.eye(2, dtype=complex)
_X = np.array([[0, 1], [1, 0]], dtype=complex)
_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z = np.array([[1, 0], [0, -1]], dtype=complex)


def popcount(v: int) -> int:
    return bin(int(v)).count("1")


def from_label(label: str):
    """``label[q]`` is the factor on qubit q, one of I X Y Z."""
    x = z = 0
    for q, ch in enumerate(label):
        if ch in "XY":
            x |= 1 << q
        if ch in "ZY":
            z |= 1 << q
        if ch not in "IXYZ":
            raise ValueError(label)
    return x, z


def to_label(x: int, z: int, n: int) -> str:
    out = []
    for q in range(n):
        bx, bz = (x >> q) & 1, (z >> q) & 1
        out.append("IZXY"[bx * 2 + bz])
    return "".join(out)


def single_factor(x: int, z: int, q: int) -> np.ndarray:
    bx, bz = (x >> q) & 1, (z >> q) & 1
    return [[_I2, _Z], [_X, _Y]][bx][bz]


def dense(x: int, z: int, n: int) -> np.ndarray:
    """Dense 2^n x 2^n matrix as a Kronecker product.  ``np.kron(A, B)`` puts
    A on the high bits, so the factor of qubit n-1 comes first."""
    m = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        m = np.kron(m, single_factor(x, z, q))
    return m


def product(x1: int, z1: int, x2: int, z2: int):
    """``P1 P2 = i^e P3``; returns ``(e mod 4, x3, z3)``.

    Moving Z^{z1} past X^{x2} gives (-1)^{|z1 & x2|}; the canonical phases
    i^{|x z|} of the two factors and of the result are accounted for."""
    x3, z3 = x1 ^ x2, z1 ^ z2
    e = popcount(x1 & z1) + popcount(x2 & z2) - popcount(x3 & z3) + 2 * popcount(z1 & x2)
    return e % 4, x3, z3


def commute(x1: int, z1: int, x2: int, z2: int) -> bool:
    return (popcount(x1 & z2) + popcount(z1 & x2)) % 2 == 0


def apply(psi: np.ndarray, x: int, z: int) -> np.ndarray:
    """``(P psi)[m] = i^{|x&z|} (-1)^{|(m^x) & z|} psi[m ^ x]``."""
    n_amp = psi.shape[0]
    m = np.arange(n_amp, dtype=np.uint64)
    src = m ^ np.uint64(x)
    sign = 1.0 - 2.0 * (np.bitwise_count(src & np.uint64(z)) & 1).astype(np.float64)
    return (1j ** (popcount(x & z) % 4)) * sign * psi[src]
