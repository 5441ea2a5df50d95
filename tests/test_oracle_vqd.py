"""Pins of the deflated (Eq. 12) energy and its reverse-mode gradient in the
oracle: finite differences, the two reductions that have closed forms, and
the excited-state energy that Eq. 12 is built to reach, against exact
diagonalization of the determinant-space Hamiltonian (no Pauli algebra)."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import fermion
from oracle import statevector as sv
from workloads import synthetic_integrals, uniform_amplitudes


def problem(n, ne, seed, excitations=None):
    h, eri = synthetic_integrals(n, seed)
    terms = fermion.jw_hamiltonian(h, eri)
    hx, hz, hc = [k[0] for k in terms], [k[1] for k in terms], list(terms.values())
    if excitations is None:
        s, d = fermion.uccsd_excitations(n, ne)
        excitations = s + d
    rots = fermion.excitation_rotations(excitations)
    return h, eri, (hx, hz, hc), rots, len(excitations)


def deflated_fg(n, ne, ham, rots, n_par, proj, alphas):
    hx, hz, hc = ham
    psi0 = sv.basis_state(n, fermion.hf_index(ne))

    def fg(th):
        e, gr = sv.deflated_reverse_gradient(psi0, hx, hz, hc, proj, alphas, [r[0] for r in rots],
                                             [r[1] for r in rots], [r[3] * th[r[2]] for r in rots])
        return e, sv.chain_to_parameters(gr, [r[2] for r in rots], [r[3] for r in rots], n_par)

    def energy(th):
        psi = sv.apply_rotations(psi0.copy(), [r[0] for r in rots], [r[1] for r in rots],
                                 [r[3] * th[r[2]] for r in rots])
        return sv.deflated_energy(psi, hx, hz, hc, proj, alphas)
    return fg, energy


def random_unit(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


def test_deflated_gradient_equals_finite_difference():
    n, ne = 6, 2
    _, _, ham, rots, n_par = problem(n, ne, 611)
    proj = [random_unit(n, 1), random_unit(n, 2)]
    fg, energy = deflated_fg(n, ne, ham, rots, n_par, proj, [0.7, 1.3])
    th = uniform_amplitudes(n_par, 0.3, 612)
    e, g = fg(th)
    assert abs(e - energy(th)) < 1e-12
    d = 1e-4
    eye = np.eye(n_par)
    for k in range(n_par):
        fd = (-energy(th + 2 * d * eye[k]) + 8 * energy(th + d * eye[k]) - 8 * energy(th - d * eye[k])
              + energy(th - 2 * d * eye[k])) / (12 * d)
        assert abs(fd - g[k]) <= 1e-9 + 1e-7 * abs(g[k]), (k, fd, g[k])
    # the deflation terms change the gradient (the pin is not the plain one)
    hx, hz, hc = ham
    _, g0 = sv.reverse_mode_gradient(sv.basis_state(n, fermion.hf_index(ne)), hx, hz, hc, [r[0] for r in rots],
                                     [r[1] for r in rots], [r[3] * th[r[2]] for r in rots])
    g0 = sv.chain_to_parameters(g0, [r[2] for r in rots], [r[3] for r in rots], n_par)
    assert np.abs(g - g0).max() > 1e-4


def test_deflation_reductions():
    """alpha = 0 is the plain Algorithm 1; deflating by the current state adds
    exactly alpha to the energy and nothing to the gradient (|<psi|psi>|^2 = 1
    for every theta)."""
    n, ne = 6, 3
    _, _, ham, rots, n_par = problem(n, ne, 621)
    hx, hz, hc = ham
    th = uniform_amplitudes(n_par, 0.4, 622)
    phis = [r[3] * th[r[2]] for r in rots]
    psi0 = sv.basis_state(n, fermion.hf_index(ne))
    e0, g0 = sv.reverse_mode_gradient(psi0, hx, hz, hc, [r[0] for r in rots], [r[1] for r in rots], phis)
    e1, g1 = sv.deflated_reverse_gradient(psi0, hx, hz, hc, [random_unit(n, 3)], [0.0], [r[0] for r in rots],
                                          [r[1] for r in rots], phis)
    assert e1 == e0 and np.array_equal(g1, g0)
    psi = sv.apply_rotations(psi0.copy(), [r[0] for r in rots], [r[1] for r in rots], phis)
    e2, g2 = sv.deflated_reverse_gradient(psi0, hx, hz, hc, [psi], [2.5], [r[0] for r in rots],
                                          [r[1] for r in rots], phis)
    assert abs(e2 - (e0 + 2.5)) < 1e-12
    assert np.abs(g2 - g0).max() < 1e-12


def test_vqd_reaches_the_first_excited_energy_at_4_qubits():
    """Two electrons in two spatial orbitals with the generalized ansatz
    (Table 1): deflating the exact ground state with alpha above the gap, the
    minimum of Eq. 12's energy is the second eigenvalue of the (N, S_z)
    sector."""
    n, ne = 4, 2
    gs, gd = fermion.uccgsd_excitations(n)
    h, eri, ham, rots, n_par = problem(n, ne, 77, excitations=gs + gd)
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    w, v = np.linalg.eigh(fermion.determinant_hamiltonian(h, eri, basis).toarray())
    ground = np.zeros(1 << n, dtype=np.complex128)
    ground[basis] = v[:, 0]
    alpha = 2.0 * (w[-1] - w[0])
    fg, _ = deflated_fg(n, ne, ham, rots, n_par, [ground], [alpha])
    best = min(minimize(fg, uniform_amplitudes(n_par, 1.0, s), jac=True, method="L-BFGS-B",
                        options={"gtol": 1e-10, "ftol": 1e-15, "maxiter": 500}).fun for s in range(4))
    assert abs(best - w[1]) < 1e-8, (best, w)
