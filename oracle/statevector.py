"""State-vector steps of the path (oracle, FP64 complex128, no fusion).

* Hartree-Fock state: the occupation bitstring of Eq. 6 (Section 3.2) as a
  basis vector.
* Rotation ``R(P, phi) = exp(-i phi P / 2) = cos(phi/2) I - i sin(phi/2) P``
  (P^2 = I).  The Trotter product of Eq. 11 is a list of these applied one at
  a time in list order; ``exp(i theta c P)`` is ``R(P, -2 c theta)``.
* Energy ``E = sum_t c_t <psi|P_t|psi>`` term by term (Eq. 2), no grouping.
* Reverse-mode differentiation, Algorithm 1 (Section 4.3), with one unitary
  per rotation ``U_k = R(P_k, phi_k)`` and ``dU_k/dphi_k = (-i/2) P_k U_k``.
* Variational quantum deflation (Section 5.1, Eq. 12): the same with H
  replaced by ``H + sum_j alpha_j |Psi_j><Psi_j|``.
"""
from __future__ import annotations

import numpy as np

from . import pauli


def basis_state(n_qubits: int, k: int) -> np.ndarray:
    psi = np.zeros(1 << n_qubits, dtype=np.complex128)
    psi[int(k)] = 1.0
    return psi


def rotate(psi: np.ndarray, x: int, z: int, phi: float) -> np.ndarray:
    return np.cos(phi / 2) * psi - 1j * np.sin(phi / 2) * pauli.apply(psi, x, z)


def apply_rotations(psi: np.ndarray, xs, zs, phis) -> np.ndarray:
    for x, z, phi in zip(xs, zs, phis):
        psi = rotate(psi, int(x), int(z), float(phi))
    return psi


def apply_hamiltonian(psi: np.ndarray, xs, zs, cs) -> np.ndarray:
    out = np.zeros_like(psi)
    for x, z, c in zip(xs, zs, cs):
        out += float(c) * pauli.apply(psi, int(x), int(z))
    return out


def expectation(psi: np.ndarray, xs, zs, cs):
    """Returns ``(sum_t c_t <psi|P_t|psi>, <psi|psi>)``; the first is complex
    (its imaginary part must vanish for a Hermitian sum)."""
    e = 0j
    for x, z, c in zip(xs, zs, cs):
        e += float(c) * np.vdot(psi, pauli.apply(psi, int(x), int(z)))
    return e, float(np.vdot(psi, psi).real)


def reverse_mode_gradient(psi0: np.ndarray, hx, hz, hc, rx, rz, rphi):
    """Algorithm 1: forward sweep, ``psi_l = H psi``, then for i from last to
    first: ``psi_r <- U_i^dag psi_r``; ``g[i] = 2 Re <psi_l| dU_i/dphi_i psi_r>``;
    ``psi_l <- U_i^dag psi_l``.  Returns ``(E, g)`` with g the derivative of
    E with respect to every rotation angle."""
    psi = apply_rotations(psi0.copy(), rx, rz, rphi)
    psi_l = apply_hamiltonian(psi, hx, hz, hc)
    return float(np.vdot(psi, psi_l).real), _backward(psi, psi_l, rx, rz, rphi)


def _backward(psi_r, psi_l, rx, rz, rphi):
    """The backward loop of Algorithm 1 from the circuit output psi_r and
    psi_l = H psi_r."""
    g = np.zeros(len(rphi))
    for i in range(len(rphi) - 1, -1, -1):
        x, z, phi = int(rx[i]), int(rz[i]), float(rphi[i])
        psi_r = rotate(psi_r, x, z, -phi)
        d_u_psi = -0.5j * pauli.apply(rotate(psi_r, x, z, phi), x, z)
        g[i] = 2.0 * np.vdot(psi_l, d_u_psi).real
        psi_l = rotate(psi_l, x, z, -phi)
    return g


def rotation_pool_gradients(psi: np.ndarray, hx, hz, hc, px, pz) -> np.ndarray:
    """Screening of Pauli rotations appended after the circuit (the Pauli
    entanglers of Section 5.1 with ADAPT): for ``R(P, tau)`` at tau = 0,
    ``dE/dtau = Im <H psi|P psi>`` (from ``dR/dtau = -i P / 2`` at 0)."""
    hpsi = apply_hamiltonian(psi, hx, hz, hc)
    return np.array([np.vdot(hpsi, pauli.apply(psi, int(x), int(z))).imag for x, z in zip(px, pz)])


def deflated_energy(psi: np.ndarray, hx, hz, hc, proj, alphas) -> float:
    """Eq. 12: ``<psi|H_eff|psi>`` with ``H_eff = H + sum_j alpha_j
    |Psi_j><Psi_j|`` (the lower states Psi_j as given), for a unit psi."""
    e, _ = expectation(psi, hx, hz, hc)
    return float(e.real) + sum(float(a) * abs(np.vdot(p, psi)) ** 2 for p, a in zip(proj, alphas))


def deflated_reverse_gradient(psi0: np.ndarray, hx, hz, hc, proj, alphas, rx, rz, rphi):
    """Algorithm 1 for the effective Hamiltonian of Eq. 12: the forward sweep,
    ``psi_l = H_eff psi = H psi + sum_j alpha_j <Psi_j|psi> Psi_j``, then the
    same backward loop.  Returns ``(<psi|H_eff|psi>, g)``."""
    psi = apply_rotations(psi0.copy(), rx, rz, rphi)
    psi_l = apply_hamiltonian(psi, hx, hz, hc)
    for p, a in zip(proj, alphas):
        psi_l = psi_l + float(a) * np.vdot(p, psi) * p
    return float(np.vdot(psi, psi_l).real), _backward(psi, psi_l, rx, rz, rphi)


def chain_to_parameters(g_rot, param_of_rot, dphi_dtheta, n_params: int) -> np.ndarray:
    """``dE/dtheta_i = sum_{k: p(k)=i} (dphi_k/dtheta_i) dE/dphi_k``."""
    out = np.zeros(n_params)
    for k, (p, d) in enumerate(zip(param_of_rot, dphi_dtheta)):
        out[int(p)] += float(d) * g_rot[k]
    return out
