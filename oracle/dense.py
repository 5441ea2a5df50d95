"""Dense-matrix cross-checks (oracle, small n only).

* ``rotation_matrix``: ``scipy.linalg.expm(-0.5j * phi * P)``.
* ``algorithm2_gates``: the circuit of Algorithm 2 (Section 5.1) for
  ``exp(i theta P)``: basis change on every non-identity factor (H for X,
  HY = (Z + Y)/sqrt(2) for Y), a CNOT chain that collects the parity of the
  support on its last qubit, ``RZ(-2 theta)`` there, then the chain and the
  basis change undone.  The printed ladder runs over all qubits with the
  parity landing on qubit 0 while RZ acts on the last qubit; the reading
  used here restricts the ladder to the support of P and chains upward into
  the highest support qubit, where RZ acts.
* ``sector_ground_energy``: exact diagonalisation in an (N, S_z) sector for
  the variational bound of Eq. 9.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import pauli

_H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
_HY = (np.array([[1, 0], [0, -1]], dtype=complex) + np.array([[0, -1j], [1j, 0]])) / np.sqrt(2)


def rz(angle: float) -> np.ndarray:
    return np.diag([np.exp(-0.5j * angle), np.exp(0.5j * angle)])


def rotation_matrix(x: int, z: int, n: int, phi: float) -> np.ndarray:
    return scipy.linalg.expm(-0.5j * phi * pauli.dense(x, z, n))


def hamiltonian_matrix(terms: dict, n: int) -> np.ndarray:
    out = np.zeros((1 << n, 1 << n), dtype=complex)
    for (x, z), c in terms.items():
        out += c * pauli.dense(x, z, n)
    return out


def algorithm2_gates(x: int, z: int, n: int, theta: float):
    """Gate list for exp(i theta P): ('1q', qubit, 2x2) or ('cx', ctrl, tgt)."""
    support = [q for q in range(n) if ((x | z) >> q) & 1]
    basis = []
    for q in support:
        bx, bz = (x >> q) & 1, (z >> q) & 1
        if bx and not bz:
            basis.append(("1q", q, _H))
        elif bx and bz:
            basis.append(("1q", q, _HY))
    ladder = [("cx", support[t], support[t + 1]) for t in range(len(support) - 1)]
    gates = list(basis) + ladder
    if support:
        gates.append(("1q", support[-1], rz(-2.0 * theta)))
    else:
        gates.append(("phase", None, np.exp(1j * theta)))
    gates += list(reversed(ladder)) + list(basis)
    return gates


def apply_gate(psi: np.ndarray, gate) -> np.ndarray:
    kind, a, b = gate
    n_amp = psi.shape[0]
    k = np.arange(n_amp)
    if kind == "phase":
        return b * psi
    if kind == "cx":
        src = np.where((k >> a) & 1, k ^ (1 << b), k)
        return psi[src]
    q, u = a, b
    bit = (k >> q) & 1
    partner = psi[k ^ (1 << q)]
    return np.where(bit == 0, u[0, 0] * psi + u[0, 1] * partner, u[1, 0] * partner + u[1, 1] * psi)


def count_cnots(gates) -> int:
    return sum(1 for g in gates if g[0] == "cx")


def sector_ground_energy(h_matrix, basis) -> float:
    sub = h_matrix[np.ix_(basis, basis)]
    return float(np.linalg.eigvalsh(sub)[0])
