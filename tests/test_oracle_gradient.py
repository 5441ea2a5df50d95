"""Pins for Algorithm 1 (reverse-mode differentiation)."""
import numpy as np

from oracle import fermion
from oracle import statevector as sv
from workloads import random_pauli_sum, random_rotations, synthetic_integrals, uniform_amplitudes


def test_algorithm1_matches_finite_differences_random():
    n = 6
    rx, rz, rphi = random_rotations(n, 12, 11, amplitude=1.0)
    hx, hz, hc = random_pauli_sum(n, 20, 12)
    psi0 = sv.basis_state(n, 0b000111)
    e, g = sv.reverse_mode_gradient(psi0, hx, hz, hc, rx, rz, rphi)

    def energy(phis):
        psi = sv.apply_rotations(psi0, rx, rz, phis)
        return sv.expectation(psi, hx, hz, hc)[0].real

    assert abs(e - energy(rphi)) < 1e-13
    for k in range(len(rphi)):
        # 4th-order central difference
        d = 1e-3
        f = lambda s: energy(np.where(np.arange(len(rphi)) == k, rphi + s, rphi))
        fd = (-f(2 * d) + 8 * f(d) - 8 * f(-d) + f(-2 * d)) / (12 * d)
        assert abs(g[k] - fd) < 1e-9


def test_gradient_at_zero_is_twice_the_hf_coupling():
    """dE/dtheta_X at theta = 0 equals 2 <HF|H tau_X|HF> (closed form)."""
    n, ne = 8, 4
    h, eri = synthetic_integrals(n, 7008)
    terms = fermion.jw_hamiltonian(h, eri)
    rots = fermion.uccsd_rotations(n, ne)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    n_par = len(singles) + len(doubles)
    hf = fermion.hf_index(ne)
    _, g = sv.reverse_mode_gradient(sv.basis_state(n, hf), [k[0] for k in terms], [k[1] for k in terms],
                                    list(terms.values()), [r[0] for r in rots], [r[1] for r in rots],
                                    np.zeros(len(rots)))
    gt = sv.chain_to_parameters(g, [r[2] for r in rots], [r[3] for r in rots], n_par)
    row = fermion.hamiltonian_on_basis_state(h, eri, hf)
    for idx, exc in enumerate(singles + doubles):
        kx, sgn = fermion.excited_determinant(exc, ne)
        assert abs(gt[idx] - 2 * sgn * row.get(kx, 0.0)) < 1e-12


def test_parameter_gradient_matches_finite_differences_uccsd():
    n, ne = 6, 3
    h, eri = synthetic_integrals(n, 8006)
    terms = fermion.jw_hamiltonian(h, eri)
    hx, hz, hc = [k[0] for k in terms], [k[1] for k in terms], list(terms.values())
    rots = fermion.uccsd_rotations(n, ne)
    n_par = max(r[2] for r in rots) + 1
    theta = uniform_amplitudes(n_par, 0.4, 5)
    psi0 = sv.basis_state(n, fermion.hf_index(ne))

    def energy(th):
        phis = [d * th[p] for _, _, p, d in rots]
        psi = sv.apply_rotations(psi0, [r[0] for r in rots], [r[1] for r in rots], phis)
        return sv.expectation(psi, hx, hz, hc)[0].real

    phis = [d * theta[p] for _, _, p, d in rots]
    _, g = sv.reverse_mode_gradient(psi0, hx, hz, hc, [r[0] for r in rots], [r[1] for r in rots], phis)
    gt = sv.chain_to_parameters(g, [r[2] for r in rots], [r[3] for r in rots], n_par)
    for i in range(n_par):
        d = 1e-3
        e = np.eye(n_par)[i]
        fd = (-energy(theta + 2 * d * e) + 8 * energy(theta + d * e) - 8 * energy(theta - d * e)
              + energy(theta - 2 * d * e)) / (12 * d)
        assert abs(gt[i] - fd) < 1e-9
