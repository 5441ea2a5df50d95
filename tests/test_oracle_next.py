"""Pins for the oracle pieces of the NEXT rows: generalized excitations
(UCCGSD, Table 1), rotation lists of any excitation sequence (Eq. 11), the
ADAPT pool gradient (Section 5.1) and the variational loop of Eq. 9."""
import itertools

import numpy as np
import pytest

from oracle import fermion
from oracle import statevector as sv
from paper_2208_10978_amd.vqe import vqe
from workloads import synthetic_integrals, uniform_amplitudes


def brute_generalized(n):
    """Every spin-conserving single and double up to the sign of its
    generator, by enumerating ordered index tuples and canonicalising."""
    spin = lambda q: q % 2
    singles, doubles = set(), set()
    for p, q in itertools.permutations(range(n), 2):
        if spin(p) == spin(q):
            singles.add(tuple(sorted((p, q))))
    for p, q, r, s in itertools.permutations(range(n), 4):
        if sorted((spin(p), spin(q))) == sorted((spin(r), spin(s))):
            a, b = tuple(sorted((p, q))), tuple(sorted((r, s)))
            doubles.add(min(a, b) + max(a, b))
    return singles, doubles


@pytest.mark.parametrize("n", [4, 6, 8])
def test_uccgsd_set_is_every_spin_conserving_operator_once(n):
    singles, doubles = fermion.uccgsd_excitations(n)
    bs, bd = brute_generalized(n)
    assert len(singles) == len(set(singles)) and set(singles) == bs
    assert len(doubles) == len(set(doubles)) and set(doubles) == bd
    m = n // 2
    assert len(singles) == 2 * m * (m - 1) // 2


@pytest.mark.parametrize("n,ne", [(4, 2), (6, 3)])
def test_generalized_rotation_list_equals_fermionic_exponentials(n, ne):
    singles, doubles = fermion.uccgsd_excitations(n)
    seq = singles + doubles
    theta = uniform_amplitudes(len(seq), 0.4, 900 + n)
    basis, phi_f = fermion.ucc_state_fermionic(n, ne, theta, excitations=seq)
    rots = fermion.excitation_rotations(seq)
    psi = sv.apply_rotations(sv.basis_state(n, fermion.hf_index(ne)), [r[0] for r in rots], [r[1] for r in rots],
                             [r[3] * theta[r[2]] for r in rots])
    assert np.abs(psi[basis] - phi_f).max() < 1e-12
    assert np.abs(psi).sum() - np.abs(psi[basis]).sum() < 1e-12


def test_pool_gradient_equals_finite_difference_of_an_appended_operator():
    n, ne = 6, 2
    h, eri = synthetic_integrals(n, 606)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    circ = singles + doubles
    theta = uniform_amplitudes(len(circ), 0.2, 707)
    gs, gd = fermion.uccgsd_excitations(n)
    pool = (gs + gd)[::7]
    g = fermion.pool_gradients(h, eri, n, ne, theta, pool, excitations=circ)
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    H = fermion.determinant_hamiltonian(h, eri, basis)

    def energy(extra, t):
        _, psi = fermion.ucc_state_fermionic(n, ne, list(theta) + [t], basis=basis, excitations=circ + [extra])
        return np.real(np.vdot(psi, H @ psi))
    d = 1e-4
    for k, op in enumerate(pool):
        fd = (-energy(op, 2 * d) + 8 * energy(op, d) - 8 * energy(op, -d) + energy(op, -2 * d)) / (12 * d)
        assert abs(fd - g[k]) <= 1e-8 + 1e-7 * abs(g[k]), (op, fd, g[k])
    assert np.abs(g).max() > 1e-3   # the screening is not trivially zero


def test_uccgsd_vqe_reaches_the_exact_ground_state_at_4_qubits():
    """Two electrons in two spatial orbitals: the four-parameter generalized
    product spans the (1 alpha, 1 beta) sector, so Eq. 9's minimum is the
    exact ground-state energy (the three-parameter UCCSD product does not
    reach it for these integrals)."""
    n, ne = 4, 2
    h, eri = synthetic_integrals(n, 77)
    basis = fermion.sector_basis(n, *fermion.electron_counts(ne))
    H = fermion.determinant_hamiltonian(h, eri, basis).toarray()
    e0 = np.linalg.eigvalsh(H)[0]
    gs, gd = fermion.uccgsd_excitations(n)
    seq = gs + gd

    def fg(th):
        def e(t):
            _, p = fermion.ucc_state_fermionic(n, ne, t, basis=basis, excitations=seq)
            return np.real(np.vdot(p, H @ p))
        eye = np.eye(len(th))
        return e(th), np.array([(e(th + 1e-6 * eye[k]) - e(th - 1e-6 * eye[k])) / 2e-6 for k in range(len(th))])
    best = min(vqe(fg, uniform_amplitudes(len(seq), 1.0, s))["energy"] for s in range(3))
    assert abs(best - e0) < 1e-9
