"""Pins for the oracle's Hamiltonian (Eq. 3 -> Eq. 1) and UCC (Eq. 10-11)."""
from math import comb

import numpy as np
import pytest
import scipy.sparse.linalg

from oracle import dense, fermion, pauli
from oracle import statevector as sv
from workloads import synthetic_integrals, uniform_amplitudes


def h_and_terms(n, seed):
    h, eri = synthetic_integrals(n, seed)
    return h, eri, fermion.jw_hamiltonian(h, eri)


@pytest.mark.parametrize("n", [4, 6, 8])
def test_jw_matrix_equals_determinant_matrix_full_space(n):
    h, eri, terms = h_and_terms(n, 1000 + n)
    hd = dense.hamiltonian_matrix(terms, n)
    hf = fermion.determinant_hamiltonian(h, eri, np.arange(1 << n)).toarray()
    assert np.abs(hd - hf).max() < 1e-12


def test_jw_matrix_equals_determinant_matrix_sector_n10():
    n = 10
    h, eri, terms = h_and_terms(n, 1010)
    basis = fermion.sector_basis(n, 3, 2)
    hf = fermion.determinant_hamiltonian(h, eri, basis).toarray()
    # apply the Pauli sum column by column to sector basis vectors
    for col in range(0, len(basis), 17):
        e = sv.basis_state(n, basis[col])
        v = sv.apply_hamiltonian(e, [k[0] for k in terms], [k[1] for k in terms], list(terms.values()))
        assert np.abs(v[basis] - hf[:, col]).max() < 1e-12
        assert np.abs(v).sum() - np.abs(v[basis]).sum() < 1e-12   # H conserves the sector


@pytest.mark.parametrize("n", [6, 8, 10])
def test_string_and_group_counts(n):
    _, _, terms = h_and_terms(n, 2000 + n)
    m = n // 2
    diag = 1 + n + comb(n, 2)
    same2 = 2 * comb(m, 2)
    mixed4 = comb(m, 2) ** 2
    same4 = 2 * comb(m, 4)
    want_strings = diag + same2 * 2 * (n - 1) + mixed4 * 4 + same4 * 6
    want_groups = 1 + same2 + mixed4 + same4
    assert len(terms) == want_strings
    assert len({k[0] for k in terms}) == want_groups


def test_hermitian_real_even_y_and_symmetries():
    n = 8
    _, _, terms = h_and_terms(n, 3008)
    for (x, z), c in terms.items():
        assert isinstance(c, float)
        assert pauli.popcount(x & z) % 2 == 0      # real symmetric strings only
    hd = dense.hamiltonian_matrix(terms, n)
    k = np.arange(1 << n)
    num = np.diag(np.bitwise_count(k).astype(float))
    sz = np.diag(np.bitwise_count(k & 0x55).astype(float) - np.bitwise_count(k & 0xAA))
    assert np.abs(hd @ num - num @ hd).max() < 1e-12
    assert np.abs(hd @ sz - sz @ hd).max() < 1e-12


@pytest.mark.parametrize("n,ne", [(4, 2), (8, 4), (10, 5), (12, 6)])
def test_hf_energy_slater_condon_equals_diagonal_terms(n, ne):
    h, eri, terms = h_and_terms(n, 4000 + n)
    k = fermion.hf_index(ne)
    diag = sum(c * (-1) ** pauli.popcount(k & z) for (x, z), c in terms.items() if x == 0)
    assert abs(diag - fermion.slater_condon_hf_energy(h, eri, ne)) < 1e-12
    row = fermion.hamiltonian_on_basis_state(h, eri, k)
    assert abs(row[k] - diag) < 1e-12


@pytest.mark.parametrize("n,ne", [(4, 2), (6, 3), (8, 4)])
def test_rotation_list_equals_fermionic_exponentials(n, ne):
    rots = fermion.uccsd_rotations(n, ne)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    n_par = len(singles) + len(doubles)
    theta = uniform_amplitudes(n_par, 0.3, 77 + n)
    psi = sv.basis_state(n, fermion.hf_index(ne))
    phis = [d * theta[p] for _, _, p, d in rots]
    psi = sv.apply_rotations(psi, [r[0] for r in rots], [r[1] for r in rots], phis)
    basis, ref = fermion.ucc_state_fermionic(n, ne, theta)
    assert np.abs(psi[basis] - ref).max() < 1e-12
    assert abs(np.linalg.norm(psi[basis]) - 1) < 1e-12


def test_rotation_list_structure():
    n, ne = 8, 4
    rots = fermion.uccsd_rotations(n, ne)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    assert len(rots) == 2 * len(singles) + 8 * len(doubles) == 160
    by_param = {}
    for x, z, p, d in rots:
        by_param.setdefault(p, []).append((x, z, d))
    for p, strings in by_param.items():
        xs = {s[0] for s in strings}
        assert len(xs) == 1                                     # one x per excitation
        mags = {abs(s[2]) for s in strings}
        assert mags == ({1.0} if len(strings) == 2 else {0.25})  # c = 1/2 or 1/8
        for (x1, z1, _), (x2, z2, _) in zip(strings, strings[1:]):
            assert pauli.commute(x1, z1, x2, z2)


def test_single_excitation_closed_form_and_slope():
    n, ne = 8, 4
    h, eri, terms = h_and_terms(n, 5008)
    singles, doubles = fermion.uccsd_excitations(n, ne)
    rots = fermion.uccsd_rotations(n, ne)
    hx = [k[0] for k in terms]; hz = [k[1] for k in terms]; hc = list(terms.values())
    hf = fermion.hf_index(ne)
    row = fermion.hamiltonian_on_basis_state(h, eri, hf)
    for target in [0, 3, len(singles) + 5]:
        exc = (singles + doubles)[target]
        kx, sgn = fermion.excited_determinant(exc, ne)
        e_hf = row[hf]
        e_x = fermion.hamiltonian_on_basis_state(h, eri, kx)[kx]
        h0x = sgn * row.get(kx, 0.0)
        for th in [0.3, -0.8]:
            theta = np.zeros(len(singles) + len(doubles)); theta[target] = th
            phis = [d * theta[p] for _, _, p, d in rots]
            psi = sv.apply_rotations(sv.basis_state(n, hf), [r[0] for r in rots], [r[1] for r in rots], phis)
            e, _ = sv.expectation(psi, hx, hz, hc)
            want = np.cos(th) ** 2 * e_hf + np.sin(th) ** 2 * e_x + 2 * np.sin(th) * np.cos(th) * h0x
            assert abs(e.real - want) < 1e-12 and abs(e.imag) < 1e-12


def test_variational_bound_n8():
    n, ne = 8, 4
    h, eri, terms = h_and_terms(n, 6008)
    hd = dense.hamiltonian_matrix(terms, n)
    basis = fermion.sector_basis(n, 2, 2)
    e0 = dense.sector_ground_energy(hd, basis)
    rots = fermion.uccsd_rotations(n, ne)
    for seed in range(3):
        theta = uniform_amplitudes(26, 0.5, seed)
        phis = [d * theta[p] for _, _, p, d in rots]
        psi = sv.apply_rotations(sv.basis_state(n, 15), [r[0] for r in rots], [r[1] for r in rots], phis)
        e, nrm = sv.expectation(psi, [k[0] for k in terms], [k[1] for k in terms], list(terms.values()))
        assert e.real >= e0 - 1e-12
        assert abs(nrm - 1) < 1e-13


@pytest.mark.parametrize("n,ne", [(4, 2), (8, 4), (12, 6), (20, 10), (26, 13), (28, 14)])
def test_tile_order_is_a_permutation(n, ne):
    from workloads import uccsd_excitation_order
    tile = uccsd_excitation_order(n, ne, "tile")
    singles, doubles = fermion.uccsd_excitations(n, ne)
    assert sorted(tile) == sorted(singles + doubles)
    assert all(len(e) == 2 for e in tile[:len(singles)])          # singles first
    assert uccsd_excitation_order(n, ne, "lex") == singles + doubles


@pytest.mark.parametrize("n,ne", [(6, 3), (8, 4)])
def test_tile_order_rotation_list_equals_fermionic_exponentials(n, ne):
    from workloads import uccsd_excitation_order
    order = uccsd_excitation_order(n, ne, "tile")
    rots = fermion.uccsd_rotations(n, ne, order)
    theta = uniform_amplitudes(len(order), 0.3, 91 + n)
    psi = sv.basis_state(n, fermion.hf_index(ne))
    psi = sv.apply_rotations(psi, [r[0] for r in rots], [r[1] for r in rots], [d * theta[p] for _, _, p, d in rots])
    basis, ref = fermion.ucc_state_fermionic(n, ne, theta, order=order)
    assert np.abs(psi[basis] - ref).max() < 1e-12


def test_order_validation():
    with pytest.raises(ValueError):
        fermion.uccsd_rotations(4, 2, [(0, 2), (1, 3)])


def test_truncate_on_a_hand_built_sum():
    """The 28-qubit workload's truncation (terms with |c| above 1e-6 kept):
    strict inequality on |c|, the sign ignored, the identity kept whatever
    its size.  Hand-built sum, expected result written out."""
    terms = {(0, 0): 1e-9,            # identity below the threshold: kept
             (0, 1): 2e-6,            # above: kept
             (0, 2): 1e-6,            # equal: dropped (strict)
             (1, 0): -3e-6,           # negative, |c| above: kept
             (1, 1): -1e-6,           # negative, equal: dropped
             (3, 0): 9.99e-7,         # just below: dropped
             (2, 2): -0.5}            # large: kept
    got = fermion.truncate(terms, 1e-6)
    assert got == {(0, 0): 1e-9, (0, 1): 2e-6, (1, 0): -3e-6, (2, 2): -0.5}
    # an identity term that is absent stays absent
    assert fermion.truncate({(1, 0): 0.1}, 1e-6) == {(1, 0): 0.1}
    assert fermion.truncate({}, 1e-6) == {}


@pytest.mark.parametrize("thr", [1e-3, 5e-3])
def test_truncation_error_is_bounded_by_the_dropped_weight(thr):
    """Dropping terms changes H by their sum, whose operator norm is at most
    the sum of their |c| (each string is unitary): checked on dense matrices
    at 8 qubits, with the removed terms recovered as full minus kept."""
    n = 8
    _, _, terms = h_and_terms(n, 1008)
    kept = fermion.truncate(terms, thr)
    dropped = {k: c for k, c in terms.items() if k not in kept}
    assert dropped and all(abs(c) <= thr for c in dropped.values())
    assert all(abs(c) > thr or k == (0, 0) for k, c in kept.items())
    diff = dense.hamiltonian_matrix(terms, n) - dense.hamiltonian_matrix(kept, n)
    assert np.abs(diff - dense.hamiltonian_matrix(dropped, n)).max() < 1e-13
    assert np.linalg.norm(diff, 2) <= sum(abs(c) for c in dropped.values()) + 1e-12
